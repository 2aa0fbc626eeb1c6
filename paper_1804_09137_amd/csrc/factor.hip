// Factorisation drivers: the dense and tile low-rank Cholesky of Sigma(theta)
// (with their tangents for the gradient), the compression pipeline, the
// solves and the handle's memory.
//
// Both variants are left-looking over tile columns j = 0 .. nt-1:
//   C(:, j) = Sigma(theta)(j.., j) - sum_{k<j} L(j.., k) L(j, k)^T
// computed by one MFMA GEMM whose epilogue generates the Matérn entries
// (Section IV, Eq. (MaternCov)), so Sigma is never stored.  Then the diagonal
// tile is factored (dense POTRF plus its inverse) and the tiles below are
//   DENSE: multiplied by L_jj^{-T}                     (dense TRSM)
//   TLR:   compressed to U V~^T at the threshold and V = L_jj^{-1} V~
//          (low-rank TRSM acts on V only, Section V).
// In the TLR case L(i, k) L(j, k)^T = U_ik (V_ik^T V_jk) U_jk^T, so the sum
// over k is W U_row^T with W_ik = U_ik (V_ik^T V_jk) (batched MFMA GEMMs) and
// U_row = [U_j0 .. U_j,j-1]: the low-rank SYRK (i = j) and GEMM (i > j)
// updates of the paper's TLR Cholesky, accumulated per tile and recompressed
// once.
#include "handle.h"

#include <array>
#include <atomic>
#include <system_error>
#include <thread>

using namespace tlrk;

namespace tlri {

thread_local char g_last_error[256] = "";

[[noreturn]] void hip_fail(hipError_t e, const char* what, const char* file, int line) {
  snprintf(g_last_error, sizeof(g_last_error), "%s (%d) in %s at %s:%d", hipGetErrorName(e), (int)e, what, file, line);
  (void)hipGetLastError();
  throw Fail{TLR_EHIP};
}

[[noreturn]] void nomem(const char* what, const char* file, int line) {
  snprintf(g_last_error, sizeof(g_last_error), "capacity exceeded: %s at %s:%d", what, file, line);
  throw Fail{TLR_ENOMEM};
}


// ---- metadata staging (pinned host -> device, one column at a time) ----
int* im_take(tlr_handle_s* h, int64_t cnt, int** dptr) {
  if (h->im_use + cnt > h->im_cap) NOMEM("int metadata");
  int* hp = h->im_h + h->im_use;
  *dptr = h->im_d + h->im_use;
  h->im_use += cnt;
  return hp;
}
int64_t* lm_take(tlr_handle_s* h, int64_t cnt, int64_t** dptr) {
  if (h->lm_use + cnt > h->lm_cap) NOMEM("offset metadata");
  int64_t* hp = h->lm_h + h->lm_use;
  *dptr = h->lm_d + h->lm_use;
  h->lm_use += cnt;
  return hp;
}
void im_push(tlr_handle_s* h, const int* hp, int* dp, int64_t cnt) {
  HIPCHK(hipMemcpyAsync(dp, hp, cnt * sizeof(int), hipMemcpyHostToDevice, h->s));
}
void lm_push(tlr_handle_s* h, const int64_t* hp, int64_t* dp, int64_t cnt) {
  HIPCHK(hipMemcpyAsync(dp, hp, cnt * sizeof(int64_t), hipMemcpyHostToDevice, h->s));
}
void meta_reset(tlr_handle_s* h) {
  // callers reset only after a synchronisation of the stream that owns the set
  h->im_use = 0;
  h->lm_use = 0;
}
void prof_harvest(tlr_handle_s* h);
void sync(tlr_handle_s* h) {
  HIPCHK(hipStreamSynchronize(h->s_main));
  if (h->s_side) HIPCHK(hipStreamSynchronize(h->s_side));
  if (h->s_diag) HIPCHK(hipStreamSynchronize(h->s_diag));
  prof_harvest(h);
}

// Issue on the side stream with the second scratch set until destroyed.
struct SideStream {
  tlr_handle_s* h;
  explicit SideStream(tlr_handle_s* hh) : h(hh) {
    swap_sets();
    h->s = h->s_side;
  }
  ~SideStream() {
    h->s = h->s_main;
    swap_sets();
  }
  void swap_sets() {
    std::swap(h->Wb, h->Wb2);
    std::swap(h->Xb, h->Xb2);
    std::swap(h->Urow, h->Urow2);
    std::swap(h->skw, h->skw2);
    std::swap(h->tw, h->tw2);
    std::swap(h->im_d, h->im2_d);
    std::swap(h->im_h, h->im2_h);
    std::swap(h->im_cap, h->im2_cap);
    std::swap(h->im_use, h->im2_use);
    std::swap(h->lm_d, h->lm2_d);
    std::swap(h->lm_h, h->lm2_h);
    std::swap(h->lm_cap, h->lm2_cap);
    std::swap(h->lm_use, h->lm2_use);
  }
};

// Issue on the diagonal-step stream until destroyed (main scratch set: only
// the diagonal factorisation's workspace is used there).
struct DiagStream {
  tlr_handle_s* h;
  explicit DiagStream(tlr_handle_s* hh) : h(hh) { h->s = h->s_diag; }
  ~DiagStream() { h->s = h->s_main; }
};

// The compression's rank read-backs: a kernel copies the ranks (and with
// info the SPD word) into fine-grained host memory and then stores a new
// sequence number there (system-scope release).
void rank_publish(tlr_handle_s* h, int n, bool info) {
  const unsigned seq = ++h->pub_seq;
  HIPCHK(launch_publish(h->qr_d, n, h->qr_hd, info ? h->info_d : nullptr, h->h_info_d, h->pub_seq_d, seq, h->s));
}

// The host waits for the last publish.  A handle with the look-ahead streams
// spins on the sequence number (the wait is on its critical path; the
// completion status of the stream itself reaches the host up to milliseconds
// late while three queues retire short kernels), checking the stream for
// errors now and then; single-stream handles, which run many to a process,
// block.
void rank_wait(tlr_handle_s* h) {
  if (!h->multi) {
    HIPCHK(hipStreamSynchronize(h->s));
    return;
  }
  const unsigned want = h->pub_seq;
  for (uint64_t it = 1;; ++it) {
    if (__atomic_load_n(h->pub_seq_h, __ATOMIC_ACQUIRE) == want) return;
    if ((it & 4095) == 0) {
      const hipError_t e = hipStreamQuery(h->s);
      if (e == hipSuccess) {
        // the stream is idle, so the publish kernel has run
        if (__atomic_load_n(h->pub_seq_h, __ATOMIC_ACQUIRE) == want) return;
        HIPCHK(hipErrorLaunchFailure);
      }
      if (e != hipErrorNotReady) HIPCHK(e);
    }
  }
}

// TLR_DEBUG timing marks of the look-ahead schedule: event id of step
// dbg_step on stream st (the report after the factorisation gives each mark's
// mean time after the previous step's end).
constexpr int kDbgMarks = 21;
void dbg_mark(tlr_handle_s* h, int id, hipStream_t st) {
  if (!h->debug || h->dbg_step < 0 || h->dbg_step >= h->nt) return;
  const size_t need = (size_t)h->nt * kDbgMarks;
  if (h->dbg_ev.size() < need) {
    const size_t old = h->dbg_ev.size();
    h->dbg_ev.resize(need, nullptr);
    for (size_t i = old; i < need; ++i) HIPCHK(hipEventCreate(&h->dbg_ev[i]));
  }
  HIPCHK(hipEventRecord(h->dbg_ev[(size_t)h->dbg_step * kDbgMarks + id], st));
}
// host time since the previous host mark, into slot id (slot 0 restarts the clock)
void dbg_host(tlr_handle_s* h, int id) {
  if (!h->debug || h->dbg_step < 0) return;
  const auto now = std::chrono::steady_clock::now();
  if (id > 0) h->dbg_host[id] += std::chrono::duration<double, std::milli>(now - h->dbg_host_last).count();
  h->dbg_host_last = now;
}
void dbg_report(tlr_handle_s* h) {
  if (!h->debug || h->dbg_ev.empty()) return;
  static const char* names[kDbgMarks] = {"main: step start (pre waited)", "main: last term done", "side: tangent tail start",
                                         "side: tangent tail done (join)", "main: factor Y launched",
                                         "main: range ranks published", "main: factor B^T launched",
                                         "main: truncation ranks published", "main: compression done",
                                         "main: diagonal step waited", "main: step end", "diag: diagonal step done",
                                         "side: next pre issued part done", "side: tangent sketch done",
                                         "side: tangent last term done", "side: diagonal tangent done",
                                         "side: rest rows waited", "main: range tasks uploaded",
                                         "main: Q1 formed", "main: truncation tasks uploaded", "main: V formed"};
  double sum[kDbgMarks] = {0};
  int cnt = 0;
  for (int j = 2; j + 3 < h->nt; ++j, ++cnt) {
    hipEvent_t ref = h->dbg_ev[(size_t)(j - 1) * kDbgMarks + 10];
    for (int id = 0; id < kDbgMarks; ++id) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ref, h->dbg_ev[(size_t)j * kDbgMarks + id]) != hipSuccess) {
        (void)hipGetLastError();
        ms = 0.f;
      }
      sum[id] += ms;
    }
  }
  if (cnt == 0) return;
  static const char* hn[8] = {"", "truncation ranks seen -> compression issued", "-> diagonal wait issued",
                              "-> triangular solves issued", "-> next step's first wait issued",
                              "-> tangent chain issued", "-> diagonal step issued", "-> factor Y launched"};
  std::fprintf(stderr, "[tlr] host ms per step (mean over %d steps):", h->nt);
  for (int id = 1; id < 8; ++id) std::fprintf(stderr, " %s %.3f;", hn[id], h->dbg_host[id] / h->nt);
  std::fprintf(stderr, "\n");
  for (double& v : h->dbg_host) v = 0.0;
  std::fprintf(stderr, "[tlr] step marks (ms after the previous step's end, mean of %d steps):\n", cnt);
  for (int id = 0; id < kDbgMarks; ++id) std::fprintf(stderr, "[tlr]   %6.3f  %s\n", sum[id] / cnt, names[id]);
}

// Make room for a group of metadata takes: when the staging buffers would
// overflow, wait for the stream that owns them (every queued copy has then
// been consumed) and recycle them.  Called before a group, never inside one.
void meta_reserve(tlr_handle_s* h, int64_t ints, int64_t longs) {
  if (h->im_use + ints <= h->im_cap && h->lm_use + longs <= h->lm_cap) return;
  if (h->debug) {
    ++h->dbg_meta_syncs;
    if (h->s == h->s_main) ++h->dbg_meta_syncs_main;
  }
  HIPCHK(hipStreamSynchronize(h->s));
  meta_reset(h);
  if (ints > h->im_cap || longs > h->lm_cap) NOMEM("metadata of one launch group");
}

// Chunks (16 columns of X) of an apply launch's tasks.
int64_t apply_chunks(const HqrTask* t, int count) {
  int64_t n = 0;
  for (int q = 0; q < count; ++q) n += (t[q].kx + kApplyCols - 1) / kApplyCols;
  return n;
}

// Work-ordered (task, chunk) list of an apply launch, staged for upload: one
// pair per chunk of X that has columns, the chunks applying the most panels
// first (with X = [I; 0] a chunk needs only the panels up to its columns), so
// that the workgroup that sets the launch time is dispatched first.
const int* apply_items(tlr_handle_s* h, const HqrTask* t, int count, int* n) {
  std::vector<std::array<int, 3>> it;   // panels, task, chunk
  for (int q = 0; q < count; ++q) {
    const int np = (std::min(t[q].m, t[q].s) + 15) / 16;
    const int nch = (t[q].kx + kApplyCols - 1) / kApplyCols;
    for (int c = 0; c < nch; ++c) it.push_back({t[q].identity ? std::min(np, c * kApplyCols / 16 + 1) : np, q, c});
  }
  std::stable_sort(it.begin(), it.end(), [](const std::array<int, 3>& a, const std::array<int, 3>& b) {
    return a[0] > b[0];
  });
  *n = (int)it.size();
  if (it.empty()) return nullptr;
  int* d;
  int* p = im_take(h, 2 * (int64_t)it.size(), &d);
  for (size_t e = 0; e < it.size(); ++e) {
    p[2 * e] = it[e][1];
    p[2 * e + 1] = it[e][2];
  }
  im_push(h, p, d, 2 * (int64_t)it.size());
  return d;
}

// ---- per-kernel-class timing: an event pair around each launch group ----
size_t prof_mark(tlr_handle_s* h) {
  if (!h->prof) return 0;
  if (h->ev_used == h->evpool.size()) {
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    h->evpool.push_back(e);
  }
  const size_t i = h->ev_used++;
  HIPCHK(hipEventRecord(h->evpool[i], h->s));
  return i;
}
void prof_add(tlr_handle_s* h, int cls, size_t e0, double flops, double bytes) {
  if (!h->prof) return;
  const size_t e1 = prof_mark(h);
  h->pend.push_back({cls, e0, e1, flops, bytes});
}
// Profiling mode 2: a column-update group runs alone.  Its stream first waits
// for the other stream's queued work, and the other stream's later work waits
// for the group, so that the group's event pair brackets only its own kernels
// (with both streams busy, a kernel's workgroups can wait for CUs held by the
// other stream's kernels, and that wait would fall between the events).
hipStream_t other_stream(tlr_handle_s* h) { return h->s == h->s_main ? h->s_side : h->s_main; }
void prof_alone_begin(tlr_handle_s* h) {
  if (h->prof != 2 || !h->s_side) return;
  HIPCHK(hipEventRecord(h->ev_px, other_stream(h)));
  HIPCHK(hipStreamWaitEvent(h->s, h->ev_px, 0));
}
void prof_alone_end(tlr_handle_s* h) {
  if (h->prof != 2 || !h->s_side) return;
  HIPCHK(hipEventRecord(h->ev_py, h->s));
  HIPCHK(hipStreamWaitEvent(other_stream(h), h->ev_py, 0));
}
// call after a stream synchronisation: folds finished pairs into the stats
void prof_harvest(tlr_handle_s* h) {
  if (!h->prof) return;
  for (const auto& p : h->pend) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, h->evpool[p.e0], h->evpool[p.e1]));
    tlr_kstat& k = h->kst[p.cls];
    k.launches += 1;
    k.ms += ms;
    k.flops += p.flops;
    k.bytes += p.bytes;
  }
  h->pend.clear();
}
// start of an API call: no event pair is open, the pool can be reused
void prof_reset_pool(tlr_handle_s* h) {
  h->pend.clear();
  h->ev_used = 0;
}

Operand op_contig(const double* base, int64_t ld, int64_t r0, int64_t c0) {
  Operand o{};
  o.base = base;
  o.ld = ld;
  o.r0 = r0;
  o.c0 = c0;
  o.layout = kContig;
  return o;
}
Operand op_contigT(const double* base, int64_t ld, int64_t r0, int64_t c0) {
  Operand o = op_contig(base, ld, r0, c0);
  o.layout = kContigT;
  return o;
}
Operand op_panels(const double* base, int64_t n, int nb, int64_t r0, int64_t c0) {
  Operand o{};
  o.base = base;
  o.n = n;
  o.nb = nb;
  o.r0 = r0;
  o.c0 = c0;
  o.layout = kPanels;
  return o;
}
GemmEpi epi_linear(double alpha, double beta) {
  GemmEpi e{};
  e.kind = kEpiLinear;
  e.alpha = alpha;
  e.beta = beta;
  return e;
}
GemmEpi epi_gen(const tlr_handle_s* h, int kind, int64_t grow0, int64_t gcol0) {
  GemmEpi e{};
  e.kind = kind;
  e.alpha = 1.0;
  e.mp = h->mp;
  e.x = h->x;
  e.y = h->y;
  e.grow0 = grow0;
  e.gcol0 = gcol0;
  return e;
}

// split-K factor for a GEMM whose output grid is small and whose K is long
int choose_splitk(const tlr_handle_s* h, int64_t M, int64_t N, int64_t K) {
  const int64_t tiles = ((M + 127) / 128) * ((N + 127) / 128);
  if (tiles >= 256 || K < 2048) return 1;
  int64_t sk = std::min<int64_t>(512 / std::max<int64_t>(tiles, 1), K / 1024);
  sk = std::max<int64_t>(1, std::min<int64_t>(sk, 32));
  while (sk > 1 && sk * M * N > h->sk_cap) --sk;
  return (int)sk;
}

// mh / nh: host copies of a hinted batch's per-item M and N.  With them the
// launch gets a flat list of the real tiles (one workgroup each) instead of
// the launch maximum's tile grid per item.  flat_tiles uploads that list into
// b (unless b has one already) and returns the number of tiles; callers may
// build it ahead of the launch, gemm builds it otherwise.
int64_t flat_tiles(tlr_handle_s* h, GemmBatch& b, int tm, int tn, const int* mh, const int* nh) {
  int64_t tot = 0;
  for (int q = 0; q < b.count; ++q) tot += ((int64_t)mh[q] + tm - 1) / tm * (((int64_t)nh[q] + tn - 1) / tn);
  if (tot == 0 || b.tile_item) return tot;
  if (h->im_use + b.count + tot <= h->im_cap - h->im_cap / 4) {   // headroom for the caller's later takes
    int* first_d;
    int* first = im_take(h, b.count + tot, &first_d);
    int* item = first + b.count;
    int64_t acc = 0;
    for (int q = 0; q < b.count; ++q) {
      first[q] = (int)acc;
      const int64_t t = ((int64_t)mh[q] + tm - 1) / tm * (((int64_t)nh[q] + tn - 1) / tn);
      for (int64_t e = 0; e < t; ++e) item[acc + e] = q;
      acc += t;
    }
    im_push(h, first, first_d, b.count + tot);
    b.tile_first = first_d;
    b.tile_item = first_d + b.count;
    b.ntiles = tot;
  }
  return tot;
}

void gemm(tlr_handle_s* h, int64_t M, int64_t N, int nseg, const GemmSeg* segs, double* C, int64_t ldc,
          const GemmEpi& ep, const GemmBatch* b, bool allow_split, int tm, int tn, const int* mh, const int* nh,
          int tag) {
  GemmBatch fb;
  if (b && mh && nh && tm && tn) {
    fb = *b;
    if (flat_tiles(h, fb, tm, tn, mh, nh) == 0) return;
    b = &fb;
  }
  int sk = 1;
  if (allow_split && !b) {
    int64_t K = 0;
    for (int i = 0; i < nseg; ++i) K += segs[i].K;
    sk = choose_splitk(h, M, N, K);
  }
  if (sk > 1) ++h->splitk_count;
  HIPCHK(launch_gemm(M, N, nseg, segs, C, ldc, ep, b, sk, sk > 1 ? h->skw : nullptr, h->s, tm, tn, tag));
}

// ---------------------------------------------------------------------------
// Tile bookkeeping of a TLR family
// ---------------------------------------------------------------------------


// kind: 1 for a factorisation, 2 for the compression of Sigma.  When the
// family's last finished pass was of the same kind, its ranks become the
// predictions for this one (theta moves little between evaluations of an
// optimisation); an interrupted pass leaves no history.
void family_reset(tlr_handle_s* h, Family& F, int kind) {
  if (F.done_kind == kind) {
    F.r1_prev.swap(F.r1);
    F.rk_prev = F.rk;
    F.dense_meas_prev.swap(F.dense_meas);
    F.hist = true;
  } else {
    F.hist = false;
  }
  std::fill(F.dense_meas.begin(), F.dense_meas.end(), 0);
  F.done_kind = 0;
  std::fill(F.rk.begin(), F.rk.end(), 0);
  std::fill(F.r1.begin(), F.r1.end(), 0);
  std::fill(F.isdense.begin(), F.isdense.end(), 0);
  std::fill(F.uoff.begin(), F.uoff.end(), 0);
  std::fill(F.voff.begin(), F.voff.end(), 0);
}

// The next pass predicts from neighbouring tiles only (used when a factor is
// computed again with FP64 products: the FP32 pass's ranks carry its rounding).
void drop_history(tlr_handle_s* h) {
  h->fam[0].done_kind = 0;
  h->fam[1].done_kind = 0;
}

// device copies of the rank and offset tables (for the solves)
void family_upload(tlr_handle_s* h, Family& F) {
  const size_t nn = (size_t)h->nt * h->nt;
  HIPCHK(hipMemcpyAsync(F.rk_d, F.rk.data(), nn * sizeof(int), hipMemcpyHostToDevice, h->s));
  HIPCHK(hipMemcpyAsync(F.uoff_d, F.uoff.data(), nn * sizeof(int64_t), hipMemcpyHostToDevice, h->s));
  HIPCHK(hipMemcpyAsync(F.voff_d, F.voff.data(), nn * sizeof(int64_t), hipMemcpyHostToDevice, h->s));
}

// (Re)allocate the TLR arena: identity block, inverses of the diagonal
// tiles, then cap doubles of tile storage.  The previous arena (if any) is
// freed first; its contents are not kept (a factorisation starts afresh).
void arena_alloc(tlr_handle_s* h, int64_t cap) {
  const int64_t nb = h->nb, nt = h->nt;
  if (h->arena) {
    sync(h);
    (void)hipFree(h->arena);
    h->bytes -= h->arena_len * (int64_t)sizeof(double);
    h->arena = nullptr;
    h->Dinv = nullptr;
  }
  h->ident_off = 0;
  h->dinv_off = pad16(nb * nb);
  h->tile_off = h->dinv_off + pad16(nt * nb * nb);
  h->tile_cap = std::max<int64_t>(cap, 0) / kAlign * kAlign;
  h->arena_len = h->tile_off + h->tile_cap;
  void* p = nullptr;
  if (hipMalloc(&p, (size_t)h->arena_len * sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    throw Fail{TLR_ENOMEM};
  }
  h->arena = (double*)p;
  h->bytes += h->arena_len * (int64_t)sizeof(double);
  h->Dinv = h->arena + h->dinv_off;
  h->tile_used = 0;
  HIPCHK(launch_fill(h->arena + h->ident_off, nb, nb, nb, 0.0, h->s));
  HIPCHK(launch_identity(h->arena + h->ident_off, nb, nb, h->s));
}

// nd doubles of tile storage (128-byte aligned); TLR_ENOMEM when the arena is full
int64_t tile_take(tlr_handle_s* h, int64_t nd) {
  const int64_t a = pad16(nd);
  if (h->tile_used + a > h->tile_cap) {
    h->tile_overflow = true;
    NOMEM("tile storage (tlr_opts.arena_bytes)");
  }
  const int64_t off = h->tile_off + h->tile_used;
  h->tile_used += a;
  return off;
}

void throw_if_not_spd(tlr_handle_s* h) {
  // *h_info was copied back before the last synchronisation
  if (*h->h_info != ~0ull) throw Fail{TLR_ENOTSPD};
}

// Rank predictions for a column: final ranks and range-finder ranks.
struct RankPred {
  std::vector<int> k, r1;
  bool hist = false;   // from the same tiles of the previous factorisation (else from neighbours)
  std::vector<char> meas;   // with history: the tile was found dense by its measured rank last time
};

// ---------------------------------------------------------------------------
// Compression of the tiles below the diagonal of one or more columns (the
// primal column j+1 and the tangent column j share every launch).  Job k's
// tiles are held densely in its src (ld = n, inside the column workspace),
// tile t being global tile i = i_first + t of column col, and occupy the
// global slots g0 .. g0 + T - 1 of the compression scratch.
// Low-rank tiles: U written to the family's slot, V~ (before the TRSM) to
// Vtmp + g*vslot, rank recorded.  Tiles whose rank would exceed maxrank are
// copied to a dense block: uoff = block, voff = dense_voff, rank = ncols
// (unless strict).  pred: predicted ranks (sketch widths, early dense
// decision).
//
//   Y = C Omega; Y = Q_y R_y (blocked Householder); t1 from R_y's column
//   tails; Q1 = Q_y[:, :t1]; B^T = C^T Q1 = Q_b R_b; R_b Pi = Q_r R_r cut at
//   k; V~ = Q_b [Q_r; 0]; U = Q1 Pi R_r[:k, :]^T.
// ---------------------------------------------------------------------------
// A column update whose rows below the diagonal tile are left to the
// compression: those tiles still owe C_i -= W_i U^T (W: the update's left
// factor, rows from the diagonal tile on, leading dimension ldw; U: the row
// factor, nb x K).  The compression applies it inside its sketch and
// projection products instead of rewriting the whole column.  A tangent
// column also owes, per tile t, its correction C_t -= Uc_t P_t^T (Uc_t the
// primal tile's left factor in the arena, P_t = dL_jj V~_t); W then holds
// Uc_t beside the term's own columns, in columns K .. K + cr[t] of the tile's
// rows, so that one product with W^T gives both parts of the projection.
struct FoldOut {
  // in (optional): where the update builds W (wld rows apart, wcols columns
  // available) and U_row
  double* wdst = nullptr;
  int64_t wld = 0;
  int wcols = 0;
  double* udst = nullptr;
  int extra = 0;                // columns of W kept after the term's own for the correction
  // out: K > 0 when the column is folded
  const double* W = nullptr;
  int64_t ldw = 0;
  const double* U = nullptr;
  int K = 0;
  const double* zs = nullptr;   // -(Omega^T U) (and -(Omega^T Pc) after it): ld smax; null: computed here
  bool corr = false;            // the per-tile correction
  std::vector<int64_t> cu;      // Uc_t: arena offset
  std::vector<int> cr;          // Uc_t: columns (0: no correction for the tile)
  std::vector<int64_t> cp;      // P_t: first column in Pc (its Omega products: column K + cp in zs)
  const double* Pc = nullptr;   // nb x (sum cr), ld nb
};

struct ColumnJob {
  const double* src;
  int i_first, T, col;
  Family* F;
  RankPred pred;
  int64_t dense_voff;
  int g0;
  hipEvent_t wait = nullptr;   // the compression stream waits for it before reading this column
  // optional: the stream that completes this column; its first sketch is
  // launched there (after the column, ahead of that stream's later work) and
  // `wait` is recorded after it
  hipStream_t sketch_stream = nullptr;
  FoldOut fold;   // K > 0: tile t still owes C -= W[(1 + t) nb rows..] U^T
};

// during[0], during[1]: host work to do while the compression's launches run,
// each called once: the first before the wait for the range ranks, the second
// before the wait for the truncation ranks (the caller calls what is left when
// no tile needed that wait).  Each host wait then costs the main stream no
// launch time: the launches that follow it are issued as soon as it ends.
void compress_columns(tlr_handle_s* h, std::vector<ColumnJob>& jobs, std::function<void()>* during = nullptr) {
  int G = 0;
  for (ColumnJob& jb : jobs) {
    jb.g0 = G;
    G += std::max(jb.T, 0);
  }
  if (G <= 0) return;
  if (G > h->gcap) throw Fail{TLR_EINVAL};
  const int nb = h->nb;
  const int ncols = nb;   // a column with tiles below its diagonal is never the ragged last one
  const int64_t ld = h->n;
  const int maxrank = h->maxrank;
  const int gc = h->gcap;
  const size_t e_c = prof_mark(h);
  double cflops = 0.0;
  const double tol = h->o.tol;
  // error budget: range finder (per-sample residual; the spectral error it
  // leaves is about that size, rarely twice it) + truncation (Frobenius norm
  // of the discarded block) <= tol in the spectral norm
  const double tol_range = 0.1 * tol;
  const double tol_trunc = 0.8 * tol;
  const bool piv = h->pivoted_trunc;
  std::chrono::steady_clock::time_point t_after_wait{};
  HqrTask* hq_fy = h->hq_h;            // factor Y (synchronised per round)
  HqrTask* hq_ay = h->hq_h + gc;       // Q1 = Q_y [I; 0]
  HqrTask* hq_fb = h->hq_h + 2 * gc;   // factor B^T
  HqrTask* hq_ab = h->hq_h + 3 * gc;   // V~ = Q_b [Q_r; 0]
  HqrTask* hq_wr = h->hq_h + 4 * gc;   // compact-WY factors of the truncation QR's reflectors
  HqrTask* hq_qr = h->hq_h + 5 * gc;   // Q_r = H_0 ... H_{k-1} [I_k; 0]
  // global slot -> job, local tile, source row offset (from the workspace base)
  std::vector<int> jof(G), tloc(G), rows(G);
  std::vector<int64_t> srow(G);
  for (int k = 0; k < (int)jobs.size(); ++k)
    for (int t = 0; t < jobs[k].T; ++t) {
      const int g = jobs[k].g0 + t;
      jof[g] = k;
      tloc[g] = t;
      rows[g] = tile_rows(h, jobs[k].i_first + t);
      srow[g] = (jobs[k].src - h->colbase) + (int64_t)t * nb;
    }
  // the pending terms of folded job k, applied to its tiles gs:
  // C_g -= W_g U^T (W_g: rows (1 + t) nb.. of W for tile t) and the
  // correction C_g -= Uc_t P_t^T
  std::vector<char> fold_done(G, 0);   // tile g has taken the pending terms
  auto fold_apply = [&](int k, const std::vector<int>& gs_in) {
    const FoldOut& fo = jobs[k].fold;
    std::vector<int> gs;
    for (int g : gs_in)
      if (!fold_done[g] && jof[g] == k) {
        fold_done[g] = 1;
        gs.push_back(g);
      }
    const int cntf = (int)gs.size();
    if (cntf == 0 || fo.K <= 0) return;
    meta_reserve(h, 2 * (int64_t)cntf, 4 * (int64_t)cntf);
    int* fm_d;
    int* fm_h = im_take(h, cntf, &fm_d);
    int* fk_d;
    int* fk_h = im_take(h, cntf, &fk_d);
    int64_t *fa_d, *fc_d, *fa1_d, *fb1_d;
    int64_t* fa_h = lm_take(h, cntf, &fa_d);
    int64_t* fc_h = lm_take(h, cntf, &fc_d);
    int64_t* fa1_h = lm_take(h, cntf, &fa1_d);
    int64_t* fb1_h = lm_take(h, cntf, &fb1_d);
    int maxm = 1, kc = 0;
    for (int q = 0; q < cntf; ++q) {
      const int g = gs[q], t = tloc[g];
      fm_h[q] = rows[g];
      fa_h[q] = (int64_t)(1 + t) * nb;
      fc_h[q] = srow[g];
      fk_h[q] = fo.corr ? fo.cr[t] : 0;
      fa1_h[q] = fo.corr ? fo.cu[t] : 0;
      fb1_h[q] = fo.corr ? fo.cp[t] * nb : 0;
      kc = std::max(kc, fk_h[q]);
      maxm = std::max(maxm, rows[g]);
    }
    im_push(h, fm_h, fm_d, 2 * (int64_t)cntf);
    lm_push(h, fa_h, fa_d, 4 * (int64_t)cntf);
    GemmSeg fs[2] = {};
    fs[0].A = op_contig(fo.W, fo.ldw, 0, 0);
    fs[0].B = op_contig(fo.U, nb, 0, 0);
    fs[0].K = fo.K;
    GemmBatch fb{};
    fb.count = cntf; fb.m_of = fm_d; fb.a_off = fa_d; fb.c_off = fc_d;
    if (fo.corr && kc > 0) {
      fs[1].A = op_contig(h->arena, nb, 0, 0);
      fs[1].B = op_contig(fo.Pc, nb, 0, 0);
      fs[1].K = kc;
      fb.a_off1 = fa1_d; fb.b_off1 = fb1_d; fb.k_of1 = fk_d;
    }
    gemm(h, maxm, ncols, (fo.corr && kc > 0) ? 2 : 1, fs, h->colbase, ld, epi_linear(-1.0, 1.0), &fb);
  };
  auto fail_rank = [&](int g) {
    h->bad_i = jobs[jof[g]].i_first + tloc[g];
    h->bad_j = jobs[jof[g]].col;
    throw Fail{TLR_ERANK};
  };
  std::vector<char> dense(G, 0), early(G, 0);
  std::vector<int> sz(G), t1(G, 0), todo;
  int rounds = 0;
  for (int g = 0; g < G; ++g) {
    const RankPred& pred = jobs[jof[g]].pred;
    const int t = tloc[g];
    // kept dense at once only when the same tile was found dense by its
    // measured rank in the previous factorisation: a prediction from the
    // neighbouring tiles would carry a dense tile on to every later tile of
    // its row, and a tile kept dense at once is measured again next time (theta
    // moves, and its rank may come back under maxrank)
    if (!h->strict && pred.hist && pred.k[t] > maxrank && pred.meas[t]) {
      dense[g] = 1;
      early[g] = 1;
      t1[g] = pred.r1[t];
      continue;
    }
    // first sketch width: the predicted range rank plus a margin (5% when it is
    // the same tile's rank in the previous factorisation, 15% when it comes
    // from neighbouring tiles) plus the 8-sample tail and slack; a sketch
    // that turns out too narrow is redone 1.3x wider
    const int margin = pred.hist ? pred.r1[t] / 20 : pred.r1[t] * 3 / 20;
    sz[g] = (int)std::min<int64_t>(h->smax, std::max<int64_t>(32, pad16(pred.r1[t] + margin + 16)));
    todo.push_back(g);
  }
  // 1-2. sketch and range rank; a tile with fewer than 8 samples beyond its
  // rank estimate is sketched again, alone, 1.3 times as wide
  // a folded job without them: Zs = -(Omega^T U) (smax x K), the sketch of
  // its pending term (one such job at a time: it takes the zst buffer)
  int nzs = 0;
  for (ColumnJob& jb : jobs) {
    if (jb.fold.K <= 0 || jb.fold.zs) continue;
    if (jb.fold.K > h->maxrank || jb.fold.corr || nzs++ > 0) throw Fail{TLR_EINVAL};
    GemmSeg zs{};
    zs.A = op_contigT(h->omega, nb, 0, 0);
    zs.B = op_contigT(jb.fold.U, nb, 0, 0);
    zs.K = ncols;
    gemm(h, h->smax, jb.fold.K, 1, &zs, h->zst, h->smax, epi_linear(-1.0, 0.0), nullptr, false, 64, 64);
    cflops += 2.0 * h->smax * (double)jb.fold.K * ncols;
    jb.fold.zs = h->zst;
  }
  bool waited = false;   // the jobs' wait events are on the stream
  while (!todo.empty()) {
    // job order (a job's tiles are sketched by one launch)
    std::stable_sort(todo.begin(), todo.end(), [&](int a, int b) { return jof[a] < jof[b]; });
    const int cnt = (int)todo.size();
    // the factor's task list is uploaded before the sketch (no upload
    // between the two launches)
    // the factor's tasks widest first (the widest tile sets the launch time)
    std::vector<int> fy(todo);
    std::stable_sort(fy.begin(), fy.end(), [&](int a, int b) { return sz[a] > sz[b]; });
    for (int q = 0; q < cnt; ++q) {
      const int g = fy[q];
      HqrTask& tk = hq_fy[q];
      tk = HqrTask{};
      tk.A = h->Ybuf + (int64_t)g * nb * h->smax;
      tk.lda = nb;
      tk.m = rows[g];
      tk.s = sz[g];
      tk.T = h->Tw + (int64_t)g * h->tw_stride;
      tk.tol = tol_range;
      tk.min_tail = 8;
      tk.rank = h->qr_d + g;
      tk.flag = h->qr_d + gc + g;
    }
    HIPCHK(hipMemcpyAsync(h->hq_d, hq_fy, cnt * sizeof(HqrTask), hipMemcpyHostToDevice, h->s));
    // Sketch of todo[sb, se).  In the first round each job's tiles get their
    // own launch after that job's wait event, so a column that is complete
    // early is sketched while another is still being finished elsewhere.
    auto sketch = [&](int sb, int se, hipStream_t on, const ColumnJob& jb) {
      const int sn = se - sb;
      const FoldOut& fold = jb.fold;
      const bool fo = fold.K > 0, co = fo && fold.corr;
      const int nsg = co ? 3 : (fo ? 2 : 1);
      // on the compression stream, which owns the set
      meta_reserve(h, (co ? 3 : 2) * (int64_t)sn, (co ? 5 : (fo ? 3 : 2)) * (int64_t)sn);
      hipStream_t own = h->s;
      h->s = on ? on : own;
      int *m_d, *n_d, *k2_d = nullptr;
      int* m_h = im_take(h, sn, &m_d);
      int* n_h = im_take(h, sn, &n_d);
      int* k2_h = co ? im_take(h, sn, &k2_d) : nullptr;
      int64_t *a_d, *c_d, *a1_d = nullptr, *a2_d = nullptr, *b2_d = nullptr;
      int64_t* a_h = lm_take(h, sn, &a_d);
      int64_t* c_h = lm_take(h, sn, &c_d);
      int64_t* a1_h = fo ? lm_take(h, sn, &a1_d) : nullptr;
      int64_t* a2_h = co ? lm_take(h, sn, &a2_d) : nullptr;
      int64_t* b2_h = co ? lm_take(h, sn, &b2_d) : nullptr;
      int maxm = 1, sw = 0, kc = 0;
      for (int q = 0; q < sn; ++q) {
        const int g = todo[sb + q], t = tloc[g];
        m_h[q] = rows[g];
        n_h[q] = sz[g];
        a_h[q] = srow[g];
        c_h[q] = (int64_t)g * nb * h->smax;
        if (fo) a1_h[q] = (int64_t)(1 + t) * nb;   // rows of W for this tile
        if (co) {
          k2_h[q] = fold.cr[t];
          a2_h[q] = fold.cu[t];
          b2_h[q] = (fold.K + fold.cp[t]) * h->smax;
          kc = std::max(kc, fold.cr[t]);
        }
        maxm = std::max(maxm, m_h[q]);
        sw = std::max(sw, sz[g]);
      }
      im_push(h, m_h, m_d, (co ? 3 : 2) * (int64_t)sn);
      lm_push(h, a_h, a_d, (co ? 5 : (fo ? 3 : 2)) * (int64_t)sn);
      // Y = C Omega, and with a fold + W (-(Omega^T U))^T = (C - W U^T) Omega,
      // with the correction also + Uc_t (-(Omega^T P_t))^T
      GemmSeg sg[3] = {};
      sg[0].A = op_contig(h->colbase, ld, 0, 0);
      sg[0].B = op_contigT(h->omega, nb, 0, 0);
      sg[0].K = ncols;
      if (fo) {
        sg[1].A = op_contig(fold.W, fold.ldw, 0, 0);
        sg[1].B = op_contig(fold.zs, h->smax, 0, 0);
        sg[1].K = fold.K;
        cflops += 2.0 * maxm * sw * (double)fold.K * sn;
      }
      if (co) {
        sg[2].A = op_contig(h->arena, nb, 0, 0);
        sg[2].B = op_contig(fold.zs, h->smax, 0, 0);
        sg[2].K = std::max(kc, 1);
        cflops += 2.0 * maxm * sw * (double)kc * sn;
      }
      // one launch of 64 x 32 tiles over all the job's tiles: a wide sketch
      // takes several workgroups side by side, so its K loop (the column,
      // plus the folded terms) is not the serial time of one wide tile
      GemmBatch bt{};
      bt.count = sn; bt.m_of = m_d; bt.n_of = n_d; bt.a_off = a_d; bt.c_off = c_d;
      bt.a_off1 = a1_d;
      if (co) {
        bt.k_of2 = k2_d;
        bt.a_off2 = a2_d;
        bt.b_off2 = b2_d;
      }
      gemm(h, maxm, sw, nsg, sg, h->Ybuf, nb, epi_linear(1.0, 0.0), &bt, false, 64, 32, m_h, n_h);
      h->s = own;
    };
    // todo is in job order: [b, e) ranges of one job each
    auto job_ranges = [&](auto&& f) {
      int b0 = 0;
      for (int k = 0; k < (int)jobs.size(); ++k) {
        int e0 = b0;
        while (e0 < cnt && jof[todo[e0]] == k) ++e0;
        f(k, b0, e0);
        b0 = e0;
      }
    };
    if (!waited) {
      // A job completed on another stream is sketched there (its metadata
      // staged in this stream's set: this stream waits for that sketch before
      // the factor, so the set is consumed before this stream recycles it).
      job_ranges([&](int k, int b0, int e0) {
        if (jobs[k].sketch_stream) {
          if (e0 > b0) sketch(b0, e0, jobs[k].sketch_stream, jobs[k]);
          HIPCHK(hipEventRecord(jobs[k].wait, jobs[k].sketch_stream));
          dbg_mark(h, 13, jobs[k].sketch_stream);
          HIPCHK(hipStreamWaitEvent(h->s, jobs[k].wait, 0));
        } else {
          if (jobs[k].wait) HIPCHK(hipStreamWaitEvent(h->s, jobs[k].wait, 0));
          if (e0 > b0) sketch(b0, e0, nullptr, jobs[k]);
        }
      });
      waited = true;
    } else {
      job_ranges([&](int k, int b0, int e0) {
        if (e0 > b0) sketch(b0, e0, nullptr, jobs[k]);
      });
    }
    if (rounds == 0) {
      dbg_mark(h, 4, h->s);
      dbg_host(h, 7);
    }
    HIPCHK(launch_hqr_factor(h->hq_d, cnt, h->s));
    rank_publish(h, 2 * gc, true);
    if (rounds == 0) dbg_mark(h, 5, h->s);
    auto h0 = std::chrono::steady_clock::now();
    if (during && during[0]) {   // the host would otherwise wait here
      during[0]();
      during[0] = nullptr;
    }
    auto h1 = std::chrono::steady_clock::now();
    rank_wait(h);   // this stream only: the other may run the next step's updates
    if (h->debug) {
      const auto h2 = std::chrono::steady_clock::now();
      h->host_ms[0] += std::chrono::duration<double, std::milli>(h1 - h0).count();
      h->host_ms[1] += std::chrono::duration<double, std::milli>(h2 - h1).count();
    }
    meta_reset(h);
    throw_if_not_spd(h);
    std::vector<int> next;
    for (int q = 0; q < cnt; ++q) {
      const int g = todo[q];
      t1[g] = h->qr_h[g];
      const double m = rows[g];
      cflops += 2.0 * m * sz[g] * ncols + 2.0 * m * sz[g] * sz[g];
      if (h->qr_h[gc + g]) {
        if (sz[g] >= h->smax) {
          if (h->strict) fail_rank(g);
          dense[g] = 1;
          continue;
        }
        sz[g] = (int)std::min<int64_t>(h->smax, pad16(sz[g] + sz[g] * 3 / 10));
        next.push_back(g);
      } else if (!h->strict && t1[g] > maxrank + maxrank / 2 + 16) {
        dense[g] = 1;  // the truncation cannot get below maxrank
      }
    }
    todo.swap(next);
    ++rounds;
  }
  if (!waited)
    for (const ColumnJob& jb : jobs)
      if (jb.wait) HIPCHK(hipStreamWaitEvent(h->s, jb.wait, 0));
  std::vector<int> lr;  // tiles still headed for a low-rank form, t1 > 0
  for (int g = 0; g < G; ++g)
    if (!dense[g] && t1[g] > 0) lr.push_back(g);
  const int L = (int)lr.size();
  std::vector<int> k2(G, 0);
  if (L > 0) {
    // Every task list and metadata array of the launches up to the truncation
    // is uploaded first: an upload is a small copy kernel, and one issued
    // between two compression launches waits for a free CU, which the other
    // stream's update GEMM may hold for hundreds of microseconds.
    // Q1 = Q_y [I_t1; 0]
    int max_kx = 0;
    for (int q = 0; q < L; ++q) {
      const int g = lr[q];
      HqrTask& tk = hq_ay[q];
      tk = HqrTask{};
      tk.A = h->Ybuf + (int64_t)g * nb * h->smax;
      tk.lda = nb;
      tk.m = rows[g];
      tk.s = sz[g];
      tk.T = h->Tw + (int64_t)g * h->tw_stride;
      tk.X = h->Q1 + (int64_t)g * nb * h->smax;
      tk.ldx = nb;
      tk.kx = t1[g];
      tk.identity = 1;
      max_kx = std::max(max_kx, tk.kx);
      cflops += 2.0 * tk.m * t1[g] * t1[g];
    }
    // B^T = Q_b R_b, widest first
    std::vector<int> fb(lr);
    std::stable_sort(fb.begin(), fb.end(), [&](int a, int b) { return t1[a] > t1[b]; });
    for (int q = 0; q < L; ++q) {
      const int g = fb[q];
      HqrTask& tk = hq_fb[q];
      tk = HqrTask{};
      tk.A = h->Bt + (int64_t)g * nb * h->smax;
      tk.lda = nb;
      tk.m = ncols;
      tk.s = t1[g];
      tk.T = h->Tw + (int64_t)g * h->tw_stride;
      if (!piv) {
        // the truncation rank and Z = R_b[:k, :]^T come with the factor
        tk.tol = tol_trunc;
        tk.trunc = 1;
        tk.rank = h->qr_d + g;
        tk.flag = h->qr_d + gc + g;
        tk.Z = h->Zb + (int64_t)g * h->smax * (maxrank + 1);
        tk.ldz = h->smax;
        tk.zcap = maxrank + 1;
      }
      cflops += 2.0 * ncols * t1[g] * t1[g];
    }
    // TLR_FLAG_PIVOTED_TRUNC: truncation by pivoted QR of R_b (t1 x t1): Z =
    // Pi R_r[:k, :]^T.  Small factors stay on chip (reflectors into the Y
    // workspace, which Q1 no longer needs; Q_r is formed afterwards); larger
    // ones are copied out and pivoted in place, Q_r into Vtmp.
    std::vector<int> big;
    int nsmall = 0;
    for (int q = 0; q < L && piv; ++q)
      if (t1[lr[q]] <= kRegQrBig) ++nsmall;
    int qs = 0, qb = nsmall;
    for (int q = 0; q < L && piv; ++q) {
      const int g = lr[q];
      const bool small = t1[g] <= kRegQrBig;
      ++h->qr_class[t1[g] <= kRegQrMax ? 0 : (small ? 1 : 2)];
      QrcpTask& tk = h->tk_h[small ? qs++ : qb++];
      tk = QrcpTask{};
      tk.m = t1[g];
      tk.q = t1[g];
      tk.tol = tol_trunc;
      tk.max_rank = maxrank + 1;
      tk.min_tail = 0;
      tk.Q = small ? nullptr : h->Vtmp + (int64_t)g * h->vslot;
      tk.ldq = nb;
      tk.tau = small ? h->Tau + (int64_t)g * kRegQrBig : nullptr;
      tk.Z = h->Zb + (int64_t)g * h->smax * (maxrank + 1);
      tk.ldz = h->smax;
      tk.rank = h->qr_d + g;
      tk.flag = h->qr_d + gc + g;
      if (small) {
        tk.Y = h->Bt + (int64_t)g * nb * h->smax;
        tk.ldy = nb;
        tk.upper = 1;
        tk.W = h->Ybuf + (int64_t)g * nb * h->smax;
        tk.ldw = nb;
      } else {
        tk.Y = h->Ybuf + (int64_t)g * nb * h->smax;
        tk.ldy = nb;
        big.push_back(g);
      }
      cflops += 4.0 * t1[g] * t1[g] * t1[g] / 3.0;
    }
    // regions 1 and 2 (Q1, B^T) in one upload, then the truncation tasks
    HIPCHK(hipMemcpyAsync(h->hq_d + gc, hq_ay, (gc + L) * sizeof(HqrTask), hipMemcpyHostToDevice, h->s));
    dbg_mark(h, 17, h->s);
    if (piv) HIPCHK(hipMemcpyAsync(h->tk_d, h->tk_h, L * sizeof(QrcpTask), hipMemcpyHostToDevice, h->s));
    const int nbg = (int)big.size();
    // Folded jobs' projections: C^T Q1 + U G (+ P_t H_t with the correction),
    // with [G; H] = -(W^T Q1) over the W rows of the tile (W holds Uc_t after
    // the term's own columns), one launch for the folded tiles of all jobs
    // (their W share one buffer and leading dimension), then one projection
    // launch per folded job.  Should [G; H] not fit its buffer, the pending
    // terms are applied to those tiles instead.
    struct FoldRange {
      int k, b, e;   // job, its tiles lr[b, e)
    };
    std::vector<FoldRange> fr;
    for (int q = 0; q < L;) {
      const int k = jof[lr[q]];
      int e = q;
      while (e < L && jof[lr[e]] == k) ++e;
      if (jobs[k].fold.K > 0) fr.push_back({k, q, e});
      q = e;
    }
    auto gm_of = [&](int q) {
      const FoldOut& f = jobs[jof[lr[q]]].fold;
      return f.K + (f.corr ? f.cr[tloc[lr[q]]] : 0);
    };
    int Kg = 1, nfq = 0;
    for (const FoldRange& r : fr)
      for (int q = r.b; q < r.e; ++q) {
        Kg = std::max(Kg, gm_of(q));
        ++nfq;
      }
    if (!fr.empty()) {
      int64_t need = 0;
      for (const FoldRange& r : fr)
        for (int q = r.b; q < r.e; ++q) need += (int64_t)Kg * t1[lr[q]];
      bool shared = true;   // every folded W in the fold buffer, one leading dimension
      for (const FoldRange& r : fr)
        shared = shared && jobs[r.k].fold.ldw == jobs[fr[0].k].fold.ldw && jobs[r.k].fold.W >= h->Wf &&
                 jobs[r.k].fold.W < h->Wf + h->wf_cap;
      if (need > h->gbuf_cap || !shared) {
        for (const FoldRange& r : fr) fold_apply(r.k, std::vector<int>(lr.begin() + r.b, lr.begin() + r.e));
        fr.clear();
        nfq = 0;
      }
    }
    const int64_t ay_chunks = apply_chunks(hq_ay, L);
    meta_reserve(h, 4 * (int64_t)L + nbg + 3 * (int64_t)nfq + 2 * ay_chunks,
                 6 * (int64_t)L + 2 * (int64_t)nbg + 4 * (int64_t)nfq);
    // projection Bt_g = C_g^T Q1_g (ncols x t1); per tile also the folded
    // segments' offsets (b1: G, a2 / b2 / k2: the correction's P_t and H_t)
    int *m_d, *n_d, *k_d, *k2_d;
    int* m_h = im_take(h, L, &m_d);
    int* n_h = im_take(h, L, &n_d);
    int* k_h = im_take(h, L, &k_d);
    int* k2_h = im_take(h, L, &k2_d);
    int64_t *a_d, *b_d, *c_d, *b1_d, *a2_d, *b2_d;
    int64_t* a_h = lm_take(h, L, &a_d);
    int64_t* b_h = lm_take(h, L, &b_d);
    int64_t* c_h = lm_take(h, L, &c_d);
    int64_t* b1_h = lm_take(h, L, &b1_d);
    int64_t* a2_h = lm_take(h, L, &a2_d);
    int64_t* b2_h = lm_take(h, L, &b2_d);
    int maxn = 1;
    for (int q = 0; q < L; ++q) {
      const int g = lr[q];
      m_h[q] = ncols;
      n_h[q] = t1[g];
      k_h[q] = rows[g];
      k2_h[q] = 0;
      a_h[q] = srow[g];                               // row offset of the tile in the workspace (contigT frame)
      b_h[q] = (int64_t)g * nb * h->smax;             // Q1 block
      c_h[q] = (int64_t)g * nb * h->smax;             // Bt block
      b1_h[q] = a2_h[q] = b2_h[q] = 0;
      maxn = std::max(maxn, n_h[q]);
      cflops += 2.0 * ncols * t1[g] * k_h[q];
    }
    int big_m = 0;
    int* nn_d = nullptr;
    int64_t *so_d = nullptr, *do_d = nullptr;
    if (nbg > 0) {
      int* nn_h = im_take(h, nbg, &nn_d);
      int64_t* so_h = lm_take(h, nbg, &so_d);
      int64_t* do_h = lm_take(h, nbg, &do_d);
      for (int q = 0; q < nbg; ++q) {
        nn_h[q] = t1[big[q]];
        so_h[q] = (int64_t)big[q] * nb * h->smax;
        do_h[q] = (int64_t)big[q] * nb * h->smax;
        big_m = std::max(big_m, nn_h[q]);
      }
      im_push(h, nn_h, nn_d, nbg);
      lm_push(h, so_h, so_d, 2 * (int64_t)nbg);
    }
    GemmBatch gbt{};   // [G; H]_q = -(W_q^T Q1_q): (K + cr) x t1 at gbuf + offset, leading dimension Kg
    int* gm_h = nullptr;
    int* gn_h = nullptr;
    if (nfq > 0) {
      int *gm_d, *gn_d, *gk_d;
      gm_h = im_take(h, nfq, &gm_d);
      gn_h = im_take(h, nfq, &gn_d);
      int* gk_h = im_take(h, nfq, &gk_d);
      int64_t *ga_d, *gb_d, *gc_d;
      int64_t* ga_h = lm_take(h, nfq, &ga_d);
      int64_t* gb_h = lm_take(h, nfq, &gb_d);
      int64_t* gc_h = lm_take(h, nfq, &gc_d);
      int64_t goff = 0;
      int i = 0;
      for (const FoldRange& r : fr) {
        const FoldOut& f = jobs[r.k].fold;
        const int64_t wofs = f.W - h->Wf;
        for (int q = r.b; q < r.e; ++q, ++i) {
          const int g = lr[q], t = tloc[g];
          gm_h[i] = gm_of(q);
          gn_h[i] = t1[g];
          gk_h[i] = rows[g];
          ga_h[i] = wofs + (int64_t)(1 + t) * nb;      // W rows of the tile
          gb_h[i] = (int64_t)g * nb * h->smax;          // Q1 block
          gc_h[i] = goff;
          b1_h[q] = goff;
          if (f.corr) {
            k2_h[q] = f.cr[t];
            a2_h[q] = f.cp[t] * nb;
            b2_h[q] = goff + f.K;
          }
          goff += (int64_t)Kg * t1[g];
          cflops += 2.0 * gm_h[i] * t1[g] * (double)rows[g] + 2.0 * ncols * t1[g] * (double)gm_h[i];
        }
      }
      im_push(h, gm_h, gm_d, 3 * (int64_t)nfq);
      lm_push(h, ga_h, ga_d, 3 * (int64_t)nfq);
      gbt.count = nfq; gbt.m_of = gm_d; gbt.n_of = gn_d; gbt.k_of = gk_d;
      gbt.a_off = ga_d; gbt.b_off = gb_d; gbt.c_off = gc_d;
      flat_tiles(h, gbt, 64, 64, gm_h, gn_h);
    }
    im_push(h, m_h, m_d, 4 * (int64_t)L);
    lm_push(h, a_h, a_d, 6 * (int64_t)L);
    // launches of the projection: one per folded job, then the other tiles
    // (ranges of lr; the non-folded ones are merged when adjacent)
    struct ProjRange {
      int k, b, e;   // k < 0: not folded
    };
    std::vector<ProjRange> pr;
    {
      size_t f = 0;
      for (int q = 0; q < L;) {
        if (f < fr.size() && fr[f].b == q) {
          pr.push_back({fr[f].k, fr[f].b, fr[f].e});
          q = fr[f].e;
          ++f;
          continue;
        }
        int e = q;
        while (e < L && !(f < fr.size() && fr[f].b == e)) ++e;
        pr.push_back({-1, q, e});
        q = e;
      }
    }
    std::vector<GemmBatch> pbt(pr.size());
    for (size_t i = 0; i < pr.size(); ++i) {
      const int b = pr[i].b;
      GemmBatch& bt = pbt[i];
      bt.count = pr[i].e - b; bt.m_of = m_d + b; bt.n_of = n_d + b; bt.k_of = k_d + b;
      bt.a_off = a_d + b; bt.b_off = b_d + b; bt.c_off = c_d + b;
      if (pr[i].k >= 0) {
        bt.b_off1 = b1_d + b;
        if (jobs[pr[i].k].fold.corr) {
          bt.a_off2 = a2_d + b; bt.b_off2 = b2_d + b; bt.k_of2 = k2_d + b;
        }
      }
      flat_tiles(h, bt, 64, 32, m_h + b, n_h + b);
    }
    int n_ay = 0;
    const int* ay_items = apply_items(h, hq_ay, L, &n_ay);
    HIPCHK(launch_hqr_apply(h->hq_d + gc, L, h->s, max_kx, ay_items, n_ay));
    dbg_mark(h, 18, h->s);
    {
      if (nfq > 0) {
        GemmSeg gs{};
        gs.A = op_contigT(h->Wf, jobs[fr[0].k].fold.ldw, 0, 0);
        gs.B = op_contigT(h->Q1, nb, 0, 0);
        gs.K = nb;
        gemm(h, Kg, maxn, 1, &gs, h->gbuf, Kg, epi_linear(-1.0, 0.0), &gbt, false, 64, 64, gm_h, gn_h);
      }
      for (size_t i = 0; i < pr.size(); ++i) {
        GemmSeg sg[3] = {};
        sg[0].A = op_contigT(h->colbase, ld, 0, 0);
        sg[0].B = op_contigT(h->Q1, nb, 0, 0);
        sg[0].K = nb;
        int nsg = 1;
        if (pr[i].k >= 0) {
          const FoldOut& f = jobs[pr[i].k].fold;
          sg[1].A = op_contig(f.U, nb, 0, 0);
          sg[1].B = op_contigT(h->gbuf, Kg, 0, 0);
          sg[1].K = f.K;
          nsg = 2;
          if (f.corr) {
            int kc = 0;
            for (int q = pr[i].b; q < pr[i].e; ++q) kc = std::max(kc, k2_h[q]);
            sg[2].A = op_contig(f.Pc, nb, 0, 0);
            sg[2].B = op_contigT(h->gbuf, Kg, 0, 0);
            sg[2].K = std::max(kc, 1);
            nsg = 3;
          }
        }
        const int b = pr[i].b;
        gemm(h, ncols, maxn, nsg, sg, h->Bt, nb, epi_linear(1.0, 0.0), &pbt[i], false, 64, 32, m_h + b, n_h + b);
      }
    }
    dbg_mark(h, 6, h->s);
    HIPCHK(launch_hqr_factor(h->hq_d + 2 * gc, L, h->s));
    if (piv) {
      if (nbg > 0) HIPCHK(launch_copy_upper(h->Bt, nb, so_d, h->Ybuf, nb, do_d, nn_d, big_m, nbg, h->s));
      HIPCHK(launch_qrcp_reg(h->tk_d, nsmall, h->s));
      HIPCHK(launch_qrcp(h->tk_d + nsmall, L - nsmall, h->s, big_m));
    }
    rank_publish(h, gc, false);
    dbg_mark(h, 7, h->s);
    auto h0 = std::chrono::steady_clock::now();
    if (during && during[1]) {
      during[1]();
      during[1] = nullptr;
    }
    auto h1 = std::chrono::steady_clock::now();
    rank_wait(h);
    dbg_host(h, 0);
    if (h->debug) {
      const auto h2 = std::chrono::steady_clock::now();
      h->host_ms[2] += std::chrono::duration<double, std::milli>(h1 - h0).count();
      h->host_ms[3] += std::chrono::duration<double, std::milli>(h2 - h1).count();
      t_after_wait = h2;
    }
    meta_reset(h);
    for (int q = 0; q < L; ++q) {
      const int g = lr[q];
      k2[g] = h->qr_h[g];
      const double m = rows[g];
      cflops += 4.0 * ncols * t1[g] * k2[g] + 2.0 * m * t1[g] * k2[g];
      if (k2[g] > maxrank) {
        if (h->strict) fail_rank(g);
        dense[g] = 1;
      }
    }
  }
  // record the outcome
  int maxk = 0, nlr = 0, ndense = 0;
  for (int g = 0; g < G; ++g) {
    const ColumnJob& jb = jobs[jof[g]];
    Family& F = *jb.F;
    const int i = jb.i_first + tloc[g];
    const size_t id = tid_of(h, i, jb.col);
    F.isdense[id] = dense[g];
    F.dense_meas[id] = dense[g] && !early[g];
    F.r1[id] = t1[g];
    if (dense[g]) {
      F.rk[id] = ncols;
      F.uoff[id] = tile_take(h, (int64_t)nb * ncols);
      F.voff[id] = jb.dense_voff;
      ++ndense;
    } else {
      F.rk[id] = k2[g];
      F.uoff[id] = k2[g] > 0 ? tile_take(h, (int64_t)nb * k2[g]) : 0;
      F.voff[id] = k2[g] > 0 ? tile_take(h, (int64_t)nb * k2[g]) : 0;
      maxk = std::max(maxk, k2[g]);
      if (k2[g] > 0) ++nlr;
    }
  }
  if (h->debug) {
    for (const ColumnJob& jb : jobs) {
      int s_max = 0, t1_max = 0, k_max = 0, nbig = 0, nd = 0;
      for (int g = jb.g0; g < jb.g0 + jb.T; ++g) {
        s_max = std::max(s_max, sz[g]);
        t1_max = std::max(t1_max, t1[g]);
        if (!dense[g]) k_max = std::max(k_max, k2[g]);
        nbig += (!dense[g] && t1[g] > kRegQrBig) ? 1 : 0;
        nd += dense[g];
      }
      std::fprintf(stderr, "[tlr] col %d%s tiles %d rounds %d sketch<=%d t1<=%d k<=%d big %d dense %d\n", jb.col,
                   jb.F == &h->fam[1] ? "'" : "", jb.T, rounds, s_max, t1_max, k_max, nbig, nd);
    }
  }
  // a folded job's dense tiles take their pending terms before they are copied
  for (int k = 0; k < (int)jobs.size() && ndense > 0; ++k) {
    if (jobs[k].fold.K <= 0) continue;
    std::vector<int> gs;
    for (int g = 0; g < G; ++g)
      if (dense[g] && jof[g] == k) gs.push_back(g);
    fold_apply(k, gs);
  }
  // 6. V~ = Q_b [Q_r; 0] and U_g = Q1_g Z_g (m_g x k_g) for the low-rank tiles
  int64_t k_chunks = 0;   // 16-column chunks of the V~ (and Q_r) applications
  for (int g = 0; g < G; ++g)
    if (!dense[g] && k2[g] > 0) k_chunks += (k2[g] + kApplyCols - 1) / kApplyCols;
  meta_reserve(h, 3 * (int64_t)nlr + 2 * (int64_t)ndense + 4 * k_chunks, 3 * (int64_t)nlr + 2 * (int64_t)ndense);
  if (nlr > 0) {
    // Q_r of the tiles pivoted on chip, from their reflectors (in the Y
    // workspace) and scalars
    int nq = 0, max_k = 0;
    for (int g = 0; g < G; ++g) {
      if (!piv || dense[g] || k2[g] == 0 || t1[g] > kRegQrBig) continue;
      HqrTask& tw = hq_wr[nq];
      tw = HqrTask{};
      tw.A = h->Ybuf + (int64_t)g * nb * h->smax;
      tw.lda = nb;
      tw.m = t1[g];
      tw.s = k2[g];
      tw.T = h->Tr + (int64_t)g * h->tr_stride;
      tw.tau = h->Tau + (int64_t)g * kRegQrBig;
      HqrTask& tq = hq_qr[nq];
      tq = tw;
      tq.tau = nullptr;
      tq.X = h->Vtmp + (int64_t)g * h->vslot;
      tq.ldx = nb;
      tq.kx = k2[g];
      tq.identity = 1;
      max_k = std::max(max_k, k2[g]);
      cflops += 4.0 * t1[g] * k2[g] * (double)k2[g];
      ++nq;
    }
    int q = 0, max_kx = 0;
    for (int g = 0; g < G; ++g) {
      if (dense[g] || k2[g] == 0) continue;
      max_kx = std::max(max_kx, k2[g]);
      HqrTask& tk = hq_ab[q++];
      tk = HqrTask{};
      tk.A = h->Bt + (int64_t)g * nb * h->smax;
      tk.lda = nb;
      tk.m = ncols;
      tk.s = t1[g];
      tk.T = h->Tw + (int64_t)g * h->tw_stride;
      tk.X = h->Vtmp + (int64_t)g * h->vslot;
      tk.ldx = nb;
      tk.kx = k2[g];
      tk.xrows = t1[g];
      tk.identity = piv ? 0 : 1;   // [Q_r; 0] (pivoted) or [I_k; 0]
    }
    // regions 3 (V~), 4 and 5 (Q_r) in one upload, before the launches
    const auto u0 = std::chrono::steady_clock::now();
    HIPCHK(hipMemcpyAsync(h->hq_d + 3 * gc, hq_ab, (nq > 0 ? 2 * (size_t)gc + nq : (size_t)nlr) * sizeof(HqrTask),
                          hipMemcpyHostToDevice, h->s));
    dbg_mark(h, 19, h->s);
    if (h->debug && t_after_wait.time_since_epoch().count() != 0) {
      h->host_ms[4] += std::chrono::duration<double, std::milli>(u0 - t_after_wait).count();
      h->host_ms[5] += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - u0).count();
    }
    int *m_d, *n_d, *k_d;
    int* m_h = im_take(h, nlr, &m_d);
    int* n_h = im_take(h, nlr, &n_d);
    int* k_h = im_take(h, nlr, &k_d);
    int64_t *a_d, *b_d, *c_d;
    int64_t* a_h = lm_take(h, nlr, &a_d);
    int64_t* b_h = lm_take(h, nlr, &b_d);
    int64_t* c_h = lm_take(h, nlr, &c_d);
    int maxm = 1;
    q = 0;
    for (int g = 0; g < G; ++g) {
      if (dense[g] || k2[g] == 0) continue;
      const ColumnJob& jb = jobs[jof[g]];
      m_h[q] = rows[g];
      n_h[q] = k2[g];
      k_h[q] = t1[g];
      a_h[q] = (int64_t)g * nb * h->smax;
      b_h[q] = (int64_t)g * h->smax * (maxrank + 1);
      c_h[q] = jb.F->uoff[tid_of(h, jb.i_first + tloc[g], jb.col)];
      maxm = std::max(maxm, m_h[q]);
      ++q;
    }
    im_push(h, m_h, m_d, 3 * (int64_t)nlr);
    lm_push(h, a_h, a_d, 3 * (int64_t)nlr);
    GemmBatch bt{};
    bt.count = nlr; bt.m_of = m_d; bt.n_of = n_d; bt.k_of = k_d; bt.a_off = a_d; bt.b_off = b_d; bt.c_off = c_d;
    flat_tiles(h, bt, 64, 32, m_h, n_h);
    int n_qr = 0, n_ab = 0;
    const int* qr_items = nq > 0 ? apply_items(h, hq_qr, nq, &n_qr) : nullptr;
    const int* ab_items = apply_items(h, hq_ab, nlr, &n_ab);
    if (nq > 0) {
      HIPCHK(launch_wy_build(h->hq_d + 4 * gc, nq, h->s, max_k));
      HIPCHK(launch_hqr_apply(h->hq_d + 5 * gc, nq, h->s, max_k, qr_items, n_qr));
    }
    HIPCHK(launch_hqr_apply(h->hq_d + 3 * gc, nlr, h->s, max_kx, ab_items, n_ab));
    dbg_mark(h, 20, h->s);
    GemmSeg sg{};
    sg.A = op_contig(h->Q1, nb, 0, 0);
    sg.B = op_contigT(h->Zb, h->smax, 0, 0);
    sg.K = h->smax;
    gemm(h, maxm, maxk, 1, &sg, h->arena, nb, epi_linear(1.0, 0.0), &bt, false, 64, 32, m_h, n_h);
    if (h->debug)
      h->host_ms[6] += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - u0).count();
  }
  // dense tiles: copy the tile into its block
  if (ndense > 0) {
    int *m_d, *k_d;
    int* m_h = im_take(h, ndense, &m_d);
    int* k_h = im_take(h, ndense, &k_d);
    int64_t *so_d, *do_d;
    int64_t* so_h = lm_take(h, ndense, &so_d);
    int64_t* do_h = lm_take(h, ndense, &do_d);
    int q = 0;
    for (int g = 0; g < G; ++g) {
      if (!dense[g]) continue;
      const ColumnJob& jb = jobs[jof[g]];
      m_h[q] = rows[g];
      k_h[q] = ncols;
      so_h[q] = srow[g];
      do_h[q] = jb.F->uoff[tid_of(h, jb.i_first + tloc[g], jb.col)];
      ++q;
    }
    im_push(h, m_h, m_d, 2 * (int64_t)ndense);
    lm_push(h, so_h, so_d, 2 * (int64_t)ndense);
    HIPCHK(launch_batched_copy(h->colbase, ld, so_d, h->arena, nb, do_d, m_d, k_d, (int64_t)nb * ncols, ndense,
                               h->s));
  }
  // algorithmic bytes: each tile read by the sketch and by the projection, and
  // its factors written (U and V at its rank, a dense tile once)
  double cbytes = 0.0;
  for (int g = 0; g < G; ++g)
    cbytes += 8.0 * (2.0 * rows[g] * ncols + (dense[g] ? (double)rows[g] * ncols : (double)(rows[g] + ncols) * k2[g]));
  prof_add(h, TLR_K_COMPRESS, e_c, cflops, cbytes);
  dbg_mark(h, 8, h->s);
  dbg_host(h, 1);
}

// V(i, col) = Dinv_col * V~_i for the low-rank tiles below the diagonal
void lowrank_trsm(tlr_handle_s* h, int col, int i_first, int T, const double* vt, Family& F) {
  if (T <= 0) return;
  std::vector<int> ts;
  for (int t = 0; t < T; ++t) {
    const size_t id = tid_of(h, i_first + t, col);
    if (!F.isdense[id] && F.rk[id] > 0) ts.push_back(t);
  }
  const int cnt = (int)ts.size();
  if (cnt == 0) return;
  // one item per 128-row block of each tile: L_jj^{-1} is lower triangular,
  // so rows [128 b, 128 b + 128) need only its first 128 (b + 1) columns
  constexpr int RB = 128;
  const int nbj = tile_rows(h, col);
  const int nrb = (nbj + RB - 1) / RB;
  const int items = cnt * nrb;
  meta_reserve(h, 3 * (int64_t)items, 3 * (int64_t)items);
  int *m_d, *n_d, *k_d;
  int* m_h = im_take(h, items, &m_d);
  int* n_h = im_take(h, items, &n_d);
  int* k_h = im_take(h, items, &k_d);
  int64_t *a_d, *b_d, *c_d;
  int64_t* a_h = lm_take(h, items, &a_d);
  int64_t* b_h = lm_take(h, items, &b_d);
  int64_t* c_h = lm_take(h, items, &c_d);
  int maxk = 0;
  double kt = 0.0;
  for (int q = 0; q < cnt; ++q) {
    const int t = ts[q];
    const size_t id = tid_of(h, i_first + t, col);
    for (int rb = 0; rb < nrb; ++rb) {
      const int e = q * nrb + rb;
      m_h[e] = std::min(RB, nbj - rb * RB);
      n_h[e] = F.rk[id];
      k_h[e] = std::min(nbj, (rb + 1) * RB);
      a_h[e] = (int64_t)rb * RB;
      b_h[e] = (int64_t)t * h->vslot;
      c_h[e] = F.voff[id] + (int64_t)rb * RB;
    }
    maxk = std::max(maxk, (int)F.rk[id]);
    kt += F.rk[id];
  }
  im_push(h, m_h, m_d, 3 * (int64_t)items);
  lm_push(h, a_h, a_d, 3 * (int64_t)items);
  GemmSeg sg{};
  sg.A = op_contig(dinv_tile(h, col), h->nb, 0, 0);
  sg.B = op_contigT(vt, h->nb, 0, 0);
  sg.K = nbj;
  GemmBatch bt{};
  bt.count = items; bt.m_of = m_d; bt.n_of = n_d; bt.k_of = k_d; bt.a_off = a_d; bt.b_off = b_d; bt.c_off = c_d;
  const size_t e_t = prof_mark(h);
  gemm(h, RB, maxk, 1, &sg, h->arena, h->nb, epi_linear(1.0, 0.0), &bt, false, 64, 32, m_h, n_h);
  prof_add(h, TLR_K_LOWRANK, e_t, 2.0 * nbj * nbj * kt, 8.0 * (2.0 * nbj * kt + (double)nbj * nbj));
}

// ---------------------------------------------------------------------------
// W-build and column GEMM of the TLR factorisation:
// C(i, j) = Gen(i, j) - sum_terms sum_k L1(i,k) L2(j,k)^T, i in [j, nt),
// L1(i,k) L2(j,k)^T = U1_ik (V1_ik^T V2_jk) U2_jk^T, written to out (row
// offset (i - j) nb, ld n).  Gen is Sigma (primal) or dSigma/dbeta (tangent).
// ---------------------------------------------------------------------------
struct LRTerm {
  const Family* Fi;   // left factor family (tiles of rows i)
  const Family* Fj;   // right factor family (tiles of row j)
};

// Column j of Sigma (or dSigma/dbeta, by epi_kind) minus the terms k in
// [kb, ke) of the left-looking sum: gen = true writes the generated block
// first, gen = false subtracts from what out already holds.  A column can so
// take most of its terms while an earlier column is still being compressed,
// and the rest afterwards.
// rest_on: the rows below the diagonal tile are updated on that stream
// (ev_rest recorded there, rest_pending set): the diagonal tile is ready
// sooner for what follows on this stream.
void tlr_column_update(tlr_handle_s* h, int j, int nterms, const LRTerm* terms, double* out, int epi_kind, int kb,
                       int ke, bool gen, FoldOut* fold = nullptr, hipStream_t rest_on = nullptr) {
  kb = std::max(kb, 0);
  ke = std::min(ke, j);
  const int nt = h->nt, nb = h->nb;
  const int nbj = tile_rows(h, j);
  // K layout: for each term, for each k < j, a segment of rank_j(k) columns
  // (the GEMM takes any K, so segments are not padded)
  std::vector<int64_t> off((size_t)nterms * std::max(j, 1));
  int64_t R = 0, Ktrue = 0;
  for (int tm = 0; tm < nterms; ++tm)
    for (int k = kb; k < ke; ++k) {
      off[(size_t)tm * j + k] = R;
      const int r = terms[tm].Fj->rk[tid_of(h, j, k)];
      R += r;
      Ktrue += r;
    }
  const size_t e_urow = prof_mark(h);
  // U_row (nb_j x R): the right factors of row j, side by side (a folded
  // tangent column builds it where its compression reads it)
  double* Ut = (fold && fold->udst) ? fold->udst : h->Urow;
  if (R > 0) {
    if (!(fold && fold->udst) && (int64_t)nb * R > h->urow_cap) NOMEM("row factor buffer");
    int cnt = 0;
    for (int tm = 0; tm < nterms; ++tm)
      for (int k = kb; k < ke; ++k)
        if (terms[tm].Fj->rk[tid_of(h, j, k)] > 0) ++cnt;
    meta_reserve(h, 2 * (int64_t)cnt, 2 * (int64_t)cnt);
    int *m_d, *k_d;
    int* m_h = im_take(h, cnt, &m_d);
    int* k_h = im_take(h, cnt, &k_d);
    int64_t *so_d, *do_d;
    int64_t* so_h = lm_take(h, cnt, &so_d);
    int64_t* do_h = lm_take(h, cnt, &do_d);
    int c = 0;
    int64_t maxe = 0;
    for (int tm = 0; tm < nterms; ++tm)
      for (int k = kb; k < ke; ++k) {
        const size_t id = tid_of(h, j, k);
        const int r = terms[tm].Fj->rk[id];
        if (r <= 0) continue;
        m_h[c] = nbj;
        k_h[c] = r;
        so_h[c] = terms[tm].Fj->uoff[id];
        do_h[c] = off[(size_t)tm * j + k] * nb;
        maxe = std::max<int64_t>(maxe, (int64_t)nbj * r);
        ++c;
      }
    im_push(h, m_h, m_d, 2 * (int64_t)cnt);
    lm_push(h, so_h, so_d, 2 * (int64_t)cnt);
    HIPCHK(launch_batched_copy(h->arena, nb, so_d, Ut, nb, do_d, m_d, k_d, maxe, cnt, h->s));
  }
  prof_add(h, TLR_K_LOWRANK, e_urow, 0.0, 16.0 * nbj * (double)Ktrue);
  // W in the fold buffer when the caller asks for a fold (one chunk, its own
  // leading dimension), else in this stream's scratch
  const bool fb = fold && fold->wdst && R > 0 && R + fold->extra <= fold->wcols;
  double* Wt = fb ? fold->wdst : h->Wb;
  const int64_t wcap = fb ? fold->wld * (int64_t)fold->wcols : h->w_cap;
  // chunks of row tiles [i0, i1) such that W and X fit
  int i0 = j;
  while (i0 < nt) {
    int i1 = i0;
    int64_t xneed = 0;
    while (i1 < nt) {
      const int64_t wrows = (int64_t)(i1 + 1 - i0) * nb;
      int64_t xadd = 0;
      for (int tm = 0; tm < nterms; ++tm)
        for (int k = kb; k < ke; ++k) {
          const int a = terms[tm].Fi->rk[tid_of(h, i1, k)];
          xadd += (int64_t)(a > h->maxrank ? nb : h->maxrank) * terms[tm].Fj->rk[tid_of(h, j, k)];
        }
      if (wrows * std::max<int64_t>(R, 1) > wcap || xneed + xadd > h->x_cap) break;
      xneed += xadd;
      ++i1;
    }
    if (i1 == i0) NOMEM("W/X workspace for one row of tiles");
    int64_t mrows = 0;
    for (int i = i0; i < i1; ++i) mrows += tile_rows(h, i);
    const int64_t ldw = fb ? fold->wld : (int64_t)(i1 - i0) * nb;
    const size_t e_w = prof_mark(h);
    double wflops = 0.0, wbytes = 0.0;
    if (R > 0) {
      const int64_t pairs = (int64_t)nterms * (i1 - i0) * j;
      meta_reserve(h, 6 * pairs, 6 * pairs);
      HIPCHK(launch_fill(Wt, ldw, (int64_t)(i1 - i0) * nb, R, 0.0, h->s));
      int64_t xoff = 0;
      // pairs grouped by the kind of the left tile: low-rank (a <= maxrank) and dense
      for (int tm = 0; tm < nterms; ++tm)
        for (int grp = 0; grp < 2; ++grp) {
          const Family& Fi = *terms[tm].Fi;
          const Family& Fj = *terms[tm].Fj;
          int cnt = 0, maxa = 1, maxb = 1;
          for (int i = i0; i < i1; ++i)
            for (int k = kb; k < ke; ++k) {
              const size_t ik = tid_of(h, i, k), jk = tid_of(h, j, k);
              const int a = Fi.rk[ik], b = Fj.rk[jk];
              if (a <= 0 || b <= 0 || (int)Fi.isdense[ik] != grp) continue;
              ++cnt;
              maxa = std::max(maxa, a);
              maxb = std::max(maxb, b);
            }
          if (cnt == 0) continue;
          int *xm_d, *xn_d, *xk_d, *wm_d, *wn_d, *wk_d;
          int* xm_h = im_take(h, cnt, &xm_d);
          int* xn_h = im_take(h, cnt, &xn_d);
          int* xk_h = im_take(h, cnt, &xk_d);
          int* wm_h = im_take(h, cnt, &wm_d);
          int* wn_h = im_take(h, cnt, &wn_d);
          int* wk_h = im_take(h, cnt, &wk_d);
          int64_t *xa_d, *xb_d, *xc_d, *wa_d, *wb_d, *wc_d;
          int64_t* xa_h = lm_take(h, cnt, &xa_d);
          int64_t* xb_h = lm_take(h, cnt, &xb_d);
          int64_t* xc_h = lm_take(h, cnt, &xc_d);
          int64_t* wa_h = lm_take(h, cnt, &wa_d);
          int64_t* wb_h = lm_take(h, cnt, &wb_d);
          int64_t* wc_h = lm_take(h, cnt, &wc_d);
          int c = 0, maxrows = 1;
          for (int i = i0; i < i1; ++i)
            for (int k = kb; k < ke; ++k) {
              const size_t ik = tid_of(h, i, k), jk = tid_of(h, j, k);
              const int a = Fi.rk[ik], b = Fj.rk[jk];
              if (a <= 0 || b <= 0 || (int)Fi.isdense[ik] != grp) continue;
              xm_h[c] = a; xn_h[c] = b; xk_h[c] = nb;
              xa_h[c] = Fi.voff[ik];
              xb_h[c] = Fj.voff[jk];
              xc_h[c] = xoff;                                  // X_ik: a x b, ld maxa
              wm_h[c] = tile_rows(h, i); wn_h[c] = b; wk_h[c] = a;
              wa_h[c] = Fi.uoff[ik];
              wb_h[c] = xoff;
              wc_h[c] = (int64_t)(i - i0) * nb + off[(size_t)tm * j + k] * ldw;
              xoff += (int64_t)maxa * b;
              maxrows = std::max(maxrows, wm_h[c]);
              wflops += 2.0 * a * b * ((double)nb + wm_h[c]);
              wbytes += 8.0 * ((double)nb * (a + b) + (double)wm_h[c] * (a + b));
              ++c;
            }
          if (xoff > h->x_cap) NOMEM("X workspace");
          im_push(h, xm_h, xm_d, 6 * (int64_t)cnt);
          lm_push(h, xa_h, xa_d, 6 * (int64_t)cnt);
          GemmSeg xs{};
          xs.A = op_contigT(h->arena, nb, 0, 0);
          xs.B = op_contigT(h->arena, nb, 0, 0);
          xs.K = nb;
          GemmBatch xb{};
          xb.count = cnt;
          xb.m_of = xm_d; xb.n_of = xn_d; xb.k_of = xk_d;
          xb.a_off = xa_d; xb.b_off = xb_d; xb.c_off = xc_d;
          gemm(h, maxa, maxb, 1, &xs, h->Xb, maxa, epi_linear(1.0, 0.0), &xb, false, grp ? 128 : 32, 32, xm_h,
               xn_h);
          GemmBatch wb{};
          wb.count = cnt;
          wb.m_of = wm_d; wb.n_of = wn_d; wb.k_of = wk_d;
          wb.a_off = wa_d; wb.b_off = wb_d; wb.c_off = wc_d;
          if (grp == 0 && maxa <= kThinMaxK) {
            // W_ik = U_ik X_ik, inner dimension a rank: a streaming kernel
            HIPCHK(launch_thin_gemm(h->arena, nb, h->Xb, maxa, Wt, ldw, wb, maxrows, maxa, maxb, h->s));
          } else {
            GemmSeg ws{};
            ws.A = op_contig(h->arena, nb, 0, 0);
            ws.B = op_contigT(h->Xb, maxa, 0, 0);
            ws.K = maxa;
            gemm(h, maxrows, maxb, 1, &ws, Wt, ldw, epi_linear(1.0, 0.0), &wb, false, 128, 32, wm_h, wn_h);
          }
        }
    }
    prof_add(h, TLR_K_LOWRANK, e_w, wflops, wbytes);
    // column GEMM with generation epilogue
    GemmSeg cs{};
    cs.A = op_contig(Wt, ldw, 0, 0);
    cs.B = op_contig(Ut, nb, 0, 0);
    cs.K = R;
    // Matern generation of the block, then C -= W U_row^T
    double* cblk = out + (int64_t)(i0 - j) * nb;
    if (gen) {
      const size_t eg = prof_mark(h);
      HIPCHK(launch_matern_block(h->mp, h->x, h->y, (int64_t)i0 * nb, mrows, (int64_t)j * nb, nbj, cblk, h->n,
                                 epi_kind == kEpiDGenMinus, h->s));
      prof_add(h, TLR_K_GEN, eg, 0.0, 8.0 * (double)mrows * nbj);
    }
    // fold: one chunk from the diagonal tile to the last row, no generation;
    // only the diagonal tile is updated here (W and U_row stay for the
    // compression); a tangent column (fold->corr) keeps fold->extra columns
    // of W after the term's own for its correction
    const bool folding = fb && !gen && i0 == j && i1 == nt && (fold->corr || R <= h->maxrank);
    const bool split = !folding && rest_on && !gen && i0 == j && i1 == nt && mrows > nbj && h->prof != 2;
    const int64_t grows = (folding || split) ? nbj : mrows;
    prof_alone_begin(h);
    const size_t e0 = prof_mark(h);
    // the diagonal tile alone (folded or split column): 64 x 64 tiles, as
    // 128 x 256 ones would leave all but a few dozen CUs idle
    const int ht = grows == nbj ? 64 : 0;
    gemm(h, grows, nbj, 1, &cs, cblk, h->n, epi_linear(-1.0, 1.0), nullptr, ht == 0, ht, ht, nullptr, nullptr,
         h->upd_tag);
    // algorithmic bytes: W and U_row read once, C read (generated) and written
    prof_add(h, TLR_K_UPDATE, e0, 2.0 * grows * nbj * (double)Ktrue,
             8.0 * ((double)grows * Ktrue + (double)nbj * Ktrue + 2.0 * (double)grows * nbj));
    prof_alone_end(h);
    if (split) {
      // the rows below on rest_on, after W (no split-K: its workspace belongs
      // to this stream); this stream's scratch stays untouched until the
      // caller has waited for ev_rest
      HIPCHK(hipEventRecord(h->ev_rw, h->s));
      HIPCHK(hipStreamWaitEvent(rest_on, h->ev_rw, 0));
      hipStream_t own = h->s;
      h->s = rest_on;
      GemmSeg rs = cs;
      rs.A = op_contig(Wt + nbj, ldw, 0, 0);
      const int64_t rrows = mrows - nbj;
      const size_t e1 = prof_mark(h);
      gemm(h, rrows, nbj, 1, &rs, cblk + nbj, h->n, epi_linear(-1.0, 1.0), nullptr, false, 0, 0, nullptr, nullptr,
           h->upd_tag);
      prof_add(h, TLR_K_UPDATE, e1, 2.0 * rrows * nbj * (double)Ktrue,
               8.0 * ((double)rrows * Ktrue + (double)nbj * Ktrue + 2.0 * (double)rrows * nbj));
      HIPCHK(hipEventRecord(h->ev_rest, h->s));
      h->s = own;
      h->rest_pending = true;
    }
    if (folding) {
      fold->W = Wt;
      fold->ldw = ldw;
      fold->U = Ut;
      fold->K = (int)R;
    }
    i0 = i1;
  }
}


// ===========================================================================
// factorisation drivers
// ===========================================================================

void reset_info(tlr_handle_s* h) {
  *h->h_info = ~0ull;
  HIPCHK(hipMemcpyAsync(h->info_d, h->h_info, sizeof(unsigned long long), hipMemcpyHostToDevice, h->s));
}


double* panel(tlr_handle_s* h, double* base, int j) { return base + panel_offset(h->n, h->nb, j); }

// Tangent of the diagonal step: C_jj = L_jj L_jj^T  =>
//   M = L_jj^{-1} dC_jj L_jj^{-T},  dL_jj = L_jj Phi(M),  tr(M) -> *trace.
// dC is read from dc (ld ldc); L_jj from L (ld ldl); dL written to out (ld ldo).
void tangent_diag(tlr_handle_s* h, int j, const double* dc, int64_t ldc, const double* L, int64_t ldl, double* out,
                  int64_t ldo) {
  const int nb = h->nb, nbj = tile_rows(h, j);
  double* T1 = h->tw + 64 * (int64_t)nb;
  double* Mj = T1 + (int64_t)nb * nb;
  const double* Di = dinv_tile(h, j);
  // The three products as batches of 64 x 64 output blocks, each with the
  // inner range its triangular factors leave: L^{-1} is lower triangular, M
  // is symmetric (its lower blocks suffice: Phi zeroes the rest), and L and
  // Phi(M) are lower triangular (so is dL; its upper blocks get K = 0).
  constexpr int TB = 64;
  const int nq = (nbj + TB - 1) / TB;
  const int nall = nq * nq, nlow = nq * (nq + 1) / 2;
  meta_reserve(h, 5 * (int64_t)(2 * nall + nlow), 3 * (int64_t)(2 * nall + nlow));
  auto blk = [&](int q) { return std::min(TB, nbj - q * TB); };
  struct Item { int m, n, k; int64_t a, b, c; };
  auto run = [&](const std::vector<Item>& it, const GemmSeg& sg, double* C, int64_t ldcc) {
    const int cnt = (int)it.size();
    int *m_d, *n_d, *k_d;
    int* m_h = im_take(h, cnt, &m_d);
    int* n_h = im_take(h, cnt, &n_d);
    int* k_h = im_take(h, cnt, &k_d);
    int64_t *a_d, *b_d, *c_d;
    int64_t* a_h = lm_take(h, cnt, &a_d);
    int64_t* b_h = lm_take(h, cnt, &b_d);
    int64_t* c_h = lm_take(h, cnt, &c_d);
    for (int q = 0; q < cnt; ++q) {
      m_h[q] = it[q].m; n_h[q] = it[q].n; k_h[q] = it[q].k;
      a_h[q] = it[q].a; b_h[q] = it[q].b; c_h[q] = it[q].c;
    }
    im_push(h, m_h, m_d, 3 * (int64_t)cnt);
    lm_push(h, a_h, a_d, 3 * (int64_t)cnt);
    GemmBatch bt{};
    bt.count = cnt; bt.m_of = m_d; bt.n_of = n_d; bt.k_of = k_d; bt.a_off = a_d; bt.b_off = b_d; bt.c_off = c_d;
    gemm(h, TB, TB, 1, &sg, C, ldcc, epi_linear(1.0, 0.0), &bt, false, TB, TB, m_h, n_h);
  };
  std::vector<Item> it;
  // T1 = L^{-1} dC: row block mt needs columns k < (mt + 1) 64 of L^{-1}
  for (int mt = 0; mt < nq; ++mt)
    for (int nt = 0; nt < nq; ++nt)
      it.push_back({blk(mt), blk(nt), std::min(nbj, (mt + 1) * TB), (int64_t)mt * TB, (int64_t)nt * TB * ldc,
                    (int64_t)mt * TB + (int64_t)nt * TB * nb});
  GemmSeg a{};
  a.A = op_contig(Di, nb, 0, 0);
  a.B = op_contigT(dc, ldc, 0, 0);
  a.K = nbj;
  run(it, a, T1, nb);
  // M = T1 L^{-T}, lower blocks: column block nt needs k < (nt + 1) 64
  it.clear();
  for (int mt = 0; mt < nq; ++mt)
    for (int nt = 0; nt <= mt; ++nt)
      it.push_back({blk(mt), blk(nt), std::min(nbj, (nt + 1) * TB), (int64_t)mt * TB, (int64_t)nt * TB,
                    (int64_t)mt * TB + (int64_t)nt * TB * nb});
  GemmSeg b{};
  b.A = op_contig(T1, nb, 0, 0);
  b.B = op_contig(Di, nb, 0, 0);
  b.K = nbj;
  run(it, b, Mj, nb);
  HIPCHK(launch_phi_trace(Mj, nb, nbj, h->scal + h->nt + j, h->s));
  // dL = L Phi(M): block (mt, nt) sums k in [nt 64, (mt + 1) 64); zero above
  it.clear();
  for (int mt = 0; mt < nq; ++mt)
    for (int nt = 0; nt < nq; ++nt) {
      const int k1 = std::min(nbj, (mt + 1) * TB), k0 = nt * TB;
      if (nt <= mt)
        it.push_back({blk(mt), blk(nt), k1 - k0, (int64_t)mt * TB + (int64_t)k0 * ldl,
                      (int64_t)nt * TB * nb + k0, (int64_t)mt * TB + (int64_t)nt * TB * ldo});
      else
        it.push_back({blk(mt), blk(nt), 0, 0, 0, (int64_t)mt * TB + (int64_t)nt * TB * ldo});
    }
  GemmSeg c{};
  c.A = op_contig(L, ldl, 0, 0);
  c.B = op_contigT(Mj, nb, 0, 0);
  c.K = nbj;
  run(it, c, out, ldo);
}

void factor_dense(tlr_handle_s* h, bool tangent) {
  const int nt = h->nt, nb = h->nb;
  const int64_t n = h->n;
  reset_info(h);
  for (int j = 0; j < nt; ++j) {
    const int nbj = tile_rows(h, j);
    const int64_t M = n - (int64_t)j * nb;
    GemmSeg sg{};
    sg.A = op_panels(h->Lp, n, nb, (int64_t)j * nb, 0);
    sg.B = op_panels(h->Lp, n, nb, (int64_t)j * nb, 0);
    sg.K = (int64_t)j * nb;
    const size_t e_u = prof_mark(h);
    gemm(h, M, nbj, 1, &sg, h->col, n, epi_gen(h, kEpiGenMinus, (int64_t)j * nb, (int64_t)j * nb), nullptr, true);
    prof_add(h, TLR_K_UPDATE, e_u, 2.0 * M * nbj * (double)sg.K,
             8.0 * ((double)M * sg.K + (double)nbj * sg.K + (double)M * nbj));
    const size_t e_d = prof_mark(h);
    HIPCHK(tile_potrf_inv(h->col, n, nbj, dinv_tile(h, j), nb, h->info_d, (int64_t)j * nb, h->tw, h->s));
    HIPCHK(launch_logdiag(h->col, n, nbj, h->scal + j, h->s));
    prof_add(h, TLR_K_DIAG, e_d, 2.0 / 3.0 * nbj * (double)nbj * nbj, 16.0 * nbj * (double)nbj);
    double* pj = panel(h, h->Lp, j);
    const int64_t ldp = n - (int64_t)j * nb;
    if (M > nbj) {
      GemmSeg ts{};
      ts.A = op_contig(h->col, n, nbj, 0);
      ts.B = op_contig(dinv_tile(h, j), nb, 0, 0);
      ts.K = nbj;
      gemm(h, M - nbj, nbj, 1, &ts, pj + nbj, ldp, epi_linear(1.0, 0.0));
    }
    HIPCHK(launch_copy_block(h->col, n, pj, ldp, nbj, nbj, h->s));
    if (!tangent) continue;
    // dC(:, j) = dSigma/dbeta(j.., j) - sum_k [dL(j.., k) L(j, k)^T + L(j.., k) dL(j, k)^T]
    GemmSeg tg[2]{};
    tg[0].A = op_panels(h->Ldp, n, nb, (int64_t)j * nb, 0);
    tg[0].B = op_panels(h->Lp, n, nb, (int64_t)j * nb, 0);
    tg[0].K = (int64_t)j * nb;
    tg[1].A = op_panels(h->Lp, n, nb, (int64_t)j * nb, 0);
    tg[1].B = op_panels(h->Ldp, n, nb, (int64_t)j * nb, 0);
    tg[1].K = (int64_t)j * nb;
    const size_t e_t = prof_mark(h);
    gemm(h, M, nbj, 2, tg, h->cold, n, epi_gen(h, kEpiDGenMinus, (int64_t)j * nb, (int64_t)j * nb), nullptr, true);
    prof_add(h, TLR_K_UPDATE, e_t, 4.0 * M * nbj * (double)tg[0].K,
             16.0 * ((double)M * tg[0].K + (double)nbj * tg[0].K) + 8.0 * M * nbj);
    double* dpj = panel(h, h->Ldp, j);
    tangent_diag(h, j, h->cold, n, pj, ldp, dpj, ldp);
    if (M > nbj) {
      // dL_below = (dC_below - L_below dL_jj^T) L_jj^{-T}
      GemmSeg u{};
      u.A = op_contig(pj + nbj, ldp, 0, 0);
      u.B = op_contig(dpj, ldp, 0, 0);
      u.K = nbj;
      gemm(h, M - nbj, nbj, 1, &u, h->cold + nbj, n, epi_linear(-1.0, 1.0));
      GemmSeg v{};
      v.A = op_contig(h->cold, n, nbj, 0);
      v.B = op_contig(dinv_tile(h, j), nb, 0, 0);
      v.K = nbj;
      gemm(h, M - nbj, nbj, 1, &v, dpj + nbj, ldp, epi_linear(1.0, 0.0));
    }
  }
}

// Rank predictions for the tiles below the diagonal of column j: the same
// tile's ranks in the previous factorisation when there is one, else the
// tile up-left on the same diagonal and the tile to the left.  The final rank
// decides a tile dense early; the range-finder rank sets the sketch width.
RankPred predict_ranks(const tlr_handle_s* h, const Family& F, int j, int T) {
  RankPred p;
  p.k.resize(T);
  p.r1.resize(T);
  p.meas.assign(T, 0);
  p.hist = F.hist;
  for (int t = 0; t < T; ++t) {
    const int i = j + 1 + t;
    if (F.hist) {
      p.k[t] = F.rk_prev[tid_of(h, i, j)];
      p.r1[t] = F.r1_prev[tid_of(h, i, j)];
      p.meas[t] = F.dense_meas_prev[tid_of(h, i, j)];
    } else if (j > 0) {
      p.k[t] = std::max(F.rk[tid_of(h, i - 1, j - 1)], F.rk[tid_of(h, i, j - 1)]);
      p.r1[t] = std::max(F.r1[tid_of(h, i - 1, j - 1)], F.r1[tid_of(h, i, j - 1)]);
    } else {
      p.k[t] = 0;
      p.r1[t] = 40;
    }
  }
  return p;
}

// Left-looking TLR Cholesky, column by column.  With the tangent, the primal
// column j+1 and the tangent column j are processed in lockstep (both need
// only the primal columns <= j and the tangent columns < j), and their tiles
// share the compression launches: half as many serial launch groups, twice
// as many tiles per launch.
// FP32-product check.  The rounding of the FP32 update products perturbs
// Sigma by E; to first order log|Sigma| moves by tr(Sigma^{-1} E), and the
// part of it that lands on diagonal tile j is bounded by
// ||D_jj^{-1}||_F ||E_jj||_F, with D_jj = L_jj L_jj^T the tile's Schur
// complement and ||E_jj||_F about u32 ||A_jj - D~_jj||_F (u32 = 2^-24, the
// update being A_jj - D~_jj).  eta = u32 sum_j ||A_jj - D~_jj||_F ||D_jj^{-1}||_F
// is the estimate compared with the log-likelihood's tolerance.  Measured on
// CPU simulations of FP32-rounded updates over Matérn fields (n 1,600-6,400,
// condition 1e1-1e6) it exceeded the actual log-likelihood change by 2x on the
// worst-conditioned field and by up to 175x on well-conditioned ones.
void fp32_check_update(tlr_handle_s* h, int j) {
  const int nb = h->nb, nbj = tile_rows(h, j);
  HIPCHK(launch_matern_block(h->mp, h->x, h->y, (int64_t)j * nb, nbj, (int64_t)j * nb, nbj, h->chk_scr, nb, false,
                             h->s));
  HIPCHK(launch_sqdiff_acc(h->chk_scr, nb, diag_tile(h, j), nb, nbj, nbj, h->chk_d + 2 * j, h->s));
}
void fp32_check_inverse(tlr_handle_s* h, int j) {
  const int nb = h->nb, nbj = tile_rows(h, j);
  // D_jj^{-1} = L_jj^{-T} L_jj^{-1}
  GemmSeg sg{};
  sg.A = op_contigT(dinv_tile(h, j), nb, 0, 0);
  sg.B = op_contigT(dinv_tile(h, j), nb, 0, 0);
  sg.K = nbj;
  gemm(h, nbj, nbj, 1, &sg, h->chk_scr, nb, epi_linear(1.0, 0.0));
  HIPCHK(launch_sqdiff_acc(h->chk_scr, nb, nullptr, 0, nbj, nbj, h->chk_d + 2 * j + 1, h->s));
}
// After a log-likelihood ll from a factor with FP32 products: eta (above)
// relative to |ll| goes to info.fp32_err_bound; true when eta exceeds half of
// the 10 tol |ll| accuracy target, i.e. the factor must be computed again
// with FP64 products.
bool fp32_check_fails(tlr_handle_s* h, double ll) {
  if (h->upd_tag != 2) {
    h->info.fp32_err_bound = 0.0;
    return false;
  }
  HIPCHK(hipMemcpyAsync(h->chk_h, h->chk_d, 2 * (size_t)h->nt * sizeof(double), hipMemcpyDeviceToHost, h->s_main));
  sync(h);
  double eta = 0.0;
  for (int j = 0; j < h->nt; ++j) eta += std::sqrt(h->chk_h[2 * j]) * std::sqrt(h->chk_h[2 * j + 1]);
  eta *= std::ldexp(1.0, -24);
  h->info.fp32_err_bound = eta / std::max(std::fabs(ll), 1e-300);
  return !(eta <= 5.0 * h->o.tol * std::fabs(ll));
}

void factor_tlr(tlr_handle_s* h, bool tangent) {
  const int nt = h->nt, nb = h->nb;
  reset_info(h);
  if (h->upd_tag == 2) HIPCHK(launch_fill(h->chk_d, 2 * nt, 2 * nt, 1, 0.0, h->s));
  family_reset(h, h->fam[0], 1);
  family_reset(h, h->fam[1], 1);
  h->tile_used = 0;
  h->tile_overflow = false;
  h->qr_class[0] = h->qr_class[1] = h->qr_class[2] = 0;
  sync(h);
  meta_reset(h);
  h->im2_use = h->lm2_use = 0;   // the side stream's staging set (idle after the sync)
  Family& P = h->fam[0];
  Family& G = h->fam[1];
  // Column buffers: with the look-ahead below, the column of step j + 1 is
  // generated and updated while step j's columns are compressed, so even and
  // odd columns take different buffers.
  const bool side = tangent && h->s_side;
  auto pbuf = [&](int j) { return (side && (j & 1)) ? h->col2 : h->col; };
  auto tbuf = [&](int j) { return (side && (j & 1)) ? h->cold2 : h->cold; };
  // generation and the terms k in [kb, ke) of primal column j
  auto primal_update = [&](int j, int kb, int ke, bool gen, FoldOut* fold = nullptr) {
    LRTerm tm{&P, &P};
    tlr_column_update(h, j, 1, &tm, pbuf(j), kEpiGenMinus, kb, ke, gen, fold);
  };
  // diagonal factorisation of primal column j
  auto primal_diag = [&](int j) {
    const int nbj = tile_rows(h, j);
    const size_t e_d = prof_mark(h);
    HIPCHK(launch_copy_block(pbuf(j), h->n, diag_tile(h, j), nb, nbj, nbj, h->s));
    if (h->upd_tag == 2) fp32_check_update(h, j);
    HIPCHK(tile_potrf_inv(diag_tile(h, j), nb, nbj, dinv_tile(h, j), nb, h->info_d, (int64_t)j * nb, h->tw, h->s));
    if (h->upd_tag == 2) fp32_check_inverse(h, j);
    HIPCHK(launch_logdiag(diag_tile(h, j), nb, nbj, h->scal + j, h->s));
    prof_add(h, TLR_K_DIAG, e_d, 2.0 / 3.0 * nbj * (double)nbj * nbj, 16.0 * nbj * (double)nbj);
  };
  auto primal_job = [&](int j) {
    const int T = nt - j - 1;
    return ColumnJob{pbuf(j) + tile_rows(h, j), j + 1, T, j, &P, predict_ranks(h, P, j, T),
                     h->dinv_off + (int64_t)j * nb * nb, 0};
  };
  // dC(:, j) = dSigma/dbeta - sum_k [dL_ik L_jk^T + L_ik dL_jk^T]; the
  // tangent of the diagonal step; dC_ij <- dC_ij - L_ij dL_jj^T (then
  // compressed: dL_ij = (that) L_jj^{-T}, low-rank V <- L_jj^{-1} V)
  auto tangent_update = [&](int j, int kb, int ke, bool gen, hipStream_t rest_on = nullptr,
                            FoldOut* fold = nullptr) {
    LRTerm tt[2] = {{&G, &P}, {&P, &G}};
    tlr_column_update(h, j, 2, tt, tbuf(j), kEpiDGenMinus, kb, ke, gen, fold, rest_on);
  };
  // Whether tangent column j's last term (beyond its diagonal tile) and its
  // correction can be left to its compression, and where their factors go:
  // W in the fold buffer's tangent part with the primal tiles' U after the
  // term's columns; U_row then the P_t side by side behind the V~ copies in
  // Ptmp; -(Omega^T [U_row P]) in zst2.  Needs every primal tile of column j
  // low-rank, and the ranks within those buffers.
  auto tangent_fold_setup = [&](int j, FoldOut& f) {
    const int T = nt - j - 1;
    if (!h->Wf || j == 0 || T <= 0 || h->upd_tag == 2) return false;
    int kc = 0;
    int64_t rsum = 0;
    for (int t = 0; t < T; ++t) {
      const size_t id = tid_of(h, j + 1 + t, j);
      if (P.isdense[id] || P.rk[id] > h->maxrank) return false;
      kc = std::max(kc, P.rk[id]);
      rsum += std::max(P.rk[id], 0);
    }
    const int64_t R = (int64_t)P.rk[tid_of(h, j, j - 1)] + G.rk[tid_of(h, j, j - 1)];
    if (R <= 0 || R + kc > h->wf_tcols || rsum > kFoldRsumMax || R + rsum > h->zst2_cols ||
        (int64_t)nb * (2 * rsum + R) > h->ptmp_cap)
      return false;
    f.wdst = h->Wf + h->wf_ld * h->wf_pcols;
    f.wld = h->wf_ld;
    f.wcols = h->wf_tcols;
    f.udst = h->Ptmp + (int64_t)nb * rsum;
    f.extra = kc;
    f.corr = true;
    return true;
  };
  // the correction below reads and writes the rows below the diagonal tile
  auto rest_wait = [&]() {
    if (!h->rest_pending) return;
    HIPCHK(hipStreamWaitEvent(h->s, h->ev_rest, 0));
    h->rest_pending = false;
  };
  auto tangent_rest = [&](int j, FoldOut* tf = nullptr) {
    const int nbj = tile_rows(h, j);
    double* cold = tbuf(j);
    double* ddj = h->Dd + (int64_t)j * nb * nb;
    const size_t e_td = prof_mark(h);
    tangent_diag(h, j, cold, h->n, diag_tile(h, j), nb, ddj, nb);
    prof_add(h, TLR_K_DIAG, e_td, 6.0 * nbj * (double)nbj * nbj, 32.0 * nbj * (double)nbj);
    dbg_mark(h, 15, h->s);
    const int T = nt - j - 1;
    if (T <= 0) return;
    if (tf && tf->K > 0) {
      // folded: the correction's factors for the compression instead of
      // dC_t -= U_t P_t^T over the column.  P_t = dL_jj V~_t for all tiles
      // (the V~_t side by side, one GEMM) behind U_row; the primal U_t into
      // W beside the last term's columns; Zs = -(Omega^T [U_row P]).
      const size_t e_c = prof_mark(h);
      double cf = 0.0;
      int64_t rsum = 0;
      int cnt = 0;
      tf->cu.assign(T, 0);
      tf->cr.assign(T, 0);
      tf->cp.assign(T, 0);
      for (int t = 0; t < T; ++t) {
        const size_t id = tid_of(h, j + 1 + t, j);
        tf->cu[t] = P.uoff[id];
        tf->cr[t] = P.rk[id];
        tf->cp[t] = rsum;
        rsum += P.rk[id];
        if (P.rk[id] > 0) ++cnt;
      }
      const int64_t R = tf->K;
      double* vcat = h->Ptmp;
      double* pcat = h->Ptmp + (int64_t)nb * (rsum + R);
      tf->Pc = pcat;
      if (cnt > 0) {
        meta_reserve(h, 4 * (int64_t)cnt, 4 * (int64_t)cnt);
        int *m_d, *k_d, *m2_d, *k2_d;
        int* m_h = im_take(h, cnt, &m_d);
        int* k_h = im_take(h, cnt, &k_d);
        int* m2_h = im_take(h, cnt, &m2_d);
        int* k2_h = im_take(h, cnt, &k2_d);
        int64_t *so_d, *do_d, *so2_d, *do2_d;
        int64_t* so_h = lm_take(h, cnt, &so_d);
        int64_t* do_h = lm_take(h, cnt, &do_d);
        int64_t* so2_h = lm_take(h, cnt, &so2_d);
        int64_t* do2_h = lm_take(h, cnt, &do2_d);
        int q = 0;
        int64_t maxe = 0, maxe2 = 0;
        for (int t = 0; t < T; ++t) {
          const size_t id = tid_of(h, j + 1 + t, j);
          if (P.rk[id] <= 0) continue;
          m_h[q] = nbj; k_h[q] = P.rk[id];
          so_h[q] = P.voff[id];
          do_h[q] = tf->cp[t] * nb;
          m2_h[q] = tile_rows(h, j + 1 + t); k2_h[q] = P.rk[id];
          so2_h[q] = P.uoff[id];
          do2_h[q] = (tf->W - h->Wf) + (int64_t)(1 + t) * nb + R * tf->ldw;
          maxe = std::max<int64_t>(maxe, (int64_t)nbj * P.rk[id]);
          maxe2 = std::max<int64_t>(maxe2, (int64_t)m2_h[q] * P.rk[id]);
          ++q;
        }
        im_push(h, m_h, m_d, 4 * (int64_t)cnt);
        lm_push(h, so_h, so_d, 4 * (int64_t)cnt);
        HIPCHK(launch_batched_copy(h->arena, nb, so_d, vcat, nb, do_d, m_d, k_d, maxe, cnt, h->s));
        HIPCHK(launch_batched_copy(h->arena, nb, so2_d, h->Wf, tf->ldw, do2_d, m2_d, k2_d, maxe2, cnt, h->s));
        GemmSeg ps{};
        ps.A = op_contig(ddj, nb, 0, 0);
        ps.B = op_contigT(vcat, nb, 0, 0);
        ps.K = nbj;
        gemm(h, nbj, rsum, 1, &ps, pcat, nb, epi_linear(1.0, 0.0), nullptr, false, 64, 64);
        cf += 2.0 * nbj * nbj * (double)rsum;
      }
      GemmSeg zs{};
      zs.A = op_contigT(h->omega, nb, 0, 0);
      zs.B = op_contigT(tf->U, nb, 0, 0);   // U_row, then P right behind it
      zs.K = nbj;
      // 64 x 64 tiles: the product is smax x (R + rsum) over K = nb, a few
      // dozen 128 x 128 tiles with a long K loop each
      gemm(h, h->smax, R + rsum, 1, &zs, h->zst2, h->smax, epi_linear(-1.0, 0.0), nullptr, false, 64, 64);
      cf += 2.0 * h->smax * (double)(R + rsum) * nbj;
      tf->zs = h->zst2;
      prof_add(h, TLR_K_LOWRANK, e_c, cf, 0.0);
      dbg_mark(h, 16, h->s);
      return;
    }
    // a fold that was set up but not taken left U_row in Ptmp, where the rows
    // below (on the diagonal-step stream) read it: wait for them first
    if (tf && tf->udst) rest_wait();
    int kmax = 0, cnt = 0;
    for (int t = 0; t < T; ++t) {
      const int r = P.rk[tid_of(h, j + 1 + t, j)];
      kmax = std::max(kmax, r);
      if (r > 0) ++cnt;
    }
    const size_t e_c = prof_mark(h);
    double cf = 0.0;
    int64_t rsum = 0;
    for (int t = 0; t < T; ++t) rsum += std::max(P.rk[tid_of(h, j + 1 + t, j)], 0);
    if (cnt > 0 && kmax <= kThinMaxK && 2 * (int64_t)nb * rsum <= h->ptmp_cap) {
      // P_t = dL_jj V_t for all tiles at once: the V_t side by side (Vcat,
      // nbj x rsum) and one GEMM, then dC_t -= U_t P_t^T streamed per tile
      double* vcat = h->Ptmp;
      double* pcat = h->Ptmp + (int64_t)nb * rsum;
      meta_reserve(h, 5 * (int64_t)cnt, 5 * (int64_t)cnt);
      int *m_d, *k_d, *n_d;
      int* m_h = im_take(h, cnt, &m_d);
      int* k_h = im_take(h, cnt, &k_d);
      int64_t *so_d, *do_d;
      int64_t* so_h = lm_take(h, cnt, &so_d);
      int64_t* do_h = lm_take(h, cnt, &do_d);
      int q = 0;
      int64_t off = 0, maxe = 0;
      std::vector<int64_t> offs((size_t)T, -1);
      for (int t = 0; t < T; ++t) {
        const size_t id = tid_of(h, j + 1 + t, j);
        if (P.rk[id] <= 0) continue;
        m_h[q] = nbj; k_h[q] = P.rk[id];
        so_h[q] = P.voff[id];
        do_h[q] = off * nb;
        offs[(size_t)t] = off;
        maxe = std::max<int64_t>(maxe, (int64_t)nbj * P.rk[id]);
        off += P.rk[id];
        ++q;
      }
      im_push(h, m_h, m_d, 2 * (int64_t)cnt);
      lm_push(h, so_h, so_d, 2 * (int64_t)cnt);
      HIPCHK(launch_batched_copy(h->arena, nb, so_d, vcat, nb, do_d, m_d, k_d, maxe, cnt, h->s));
      GemmSeg ps{};
      ps.A = op_contig(ddj, nb, 0, 0);
      ps.B = op_contigT(vcat, nb, 0, 0);
      ps.K = nbj;
      // 64 x 64 tiles: the product is nbj x rsum, under 200 tiles of 128 x 128
      gemm(h, nbj, rsum, 1, &ps, pcat, nb, epi_linear(1.0, 0.0), nullptr, false, 64, 64);
      cf += 2.0 * nbj * nbj * (double)rsum;
      int* m2_h = im_take(h, cnt, &m_d);
      int* n2_h = im_take(h, cnt, &n_d);
      int* k2_h = im_take(h, cnt, &k_d);
      int64_t *a_d, *b_d, *c_d;
      int64_t* a2_h = lm_take(h, cnt, &a_d);
      int64_t* b2_h = lm_take(h, cnt, &b_d);
      int64_t* c2_h = lm_take(h, cnt, &c_d);
      int mmax = 1;
      q = 0;
      for (int t = 0; t < T; ++t) {
        const size_t id = tid_of(h, j + 1 + t, j);
        if (P.rk[id] <= 0) continue;
        m2_h[q] = tile_rows(h, j + 1 + t); n2_h[q] = nbj; k2_h[q] = P.rk[id];
        a2_h[q] = P.uoff[id];
        b2_h[q] = offs[(size_t)t] * nb;
        c2_h[q] = (int64_t)nbj + (int64_t)t * nb;
        mmax = std::max(mmax, m2_h[q]);
        cf += 2.0 * m2_h[q] * nbj * P.rk[id];
        ++q;
      }
      im_push(h, m2_h, m_d, 3 * (int64_t)cnt);
      lm_push(h, a2_h, a_d, 3 * (int64_t)cnt);
      GemmBatch cb{};
      cb.count = cnt; cb.m_of = m_d; cb.n_of = n_d; cb.k_of = k_d; cb.a_off = a_d; cb.b_off = b_d; cb.c_off = c_d;
      rest_wait();
      dbg_mark(h, 16, h->s);
      HIPCHK(launch_thin_gemm(h->arena, nb, pcat, nb, cold, h->n, cb, mmax, kmax, nbj, h->s, -1.0, 1.0, true));
    } else if (cnt > 0) {
      meta_reserve(h, 6 * (int64_t)cnt, 6 * (int64_t)cnt);
      int *m_d, *n_d, *k_d;
      int* m_h = im_take(h, cnt, &m_d);
      int* n_h = im_take(h, cnt, &n_d);
      int* k_h = im_take(h, cnt, &k_d);
      int64_t *a_d, *b_d, *c_d;
      int64_t* a_h = lm_take(h, cnt, &a_d);
      int64_t* b_h = lm_take(h, cnt, &b_d);
      int64_t* c_h = lm_take(h, cnt, &c_d);
      int q = 0;
      for (int t = 0; t < T; ++t) {
        const size_t id = tid_of(h, j + 1 + t, j);
        if (P.rk[id] <= 0) continue;
        m_h[q] = nbj; n_h[q] = P.rk[id]; k_h[q] = nbj;
        a_h[q] = 0;
        b_h[q] = P.voff[id];
        c_h[q] = (int64_t)t * nb * nb;
        cf += 2.0 * nbj * nbj * P.rk[id];
        ++q;
      }
      im_push(h, m_h, m_d, 3 * (int64_t)cnt);
      lm_push(h, a_h, a_d, 3 * (int64_t)cnt);
      GemmSeg ps{};
      ps.A = op_contig(ddj, nb, 0, 0);
      ps.B = op_contigT(h->arena, nb, 0, 0);
      ps.K = nbj;
      GemmBatch pb{};
      pb.count = cnt; pb.m_of = m_d; pb.n_of = n_d; pb.k_of = k_d; pb.a_off = a_d; pb.b_off = b_d; pb.c_off = c_d;
      gemm(h, nbj, kmax, 1, &ps, h->Ptmp, nb, epi_linear(1.0, 0.0), &pb, false, 128, kmax > 64 ? 128 : 32, m_h,
           n_h);
      int* m2_h = im_take(h, cnt, &m_d);
      int* n2_h = im_take(h, cnt, &n_d);
      int* k2_h = im_take(h, cnt, &k_d);
      int64_t* a2_h = lm_take(h, cnt, &a_d);
      int64_t* b2_h = lm_take(h, cnt, &b_d);
      int64_t* c2_h = lm_take(h, cnt, &c_d);
      int mmax = 1;
      q = 0;
      for (int t = 0; t < T; ++t) {
        const size_t id = tid_of(h, j + 1 + t, j);
        if (P.rk[id] <= 0) continue;
        m2_h[q] = tile_rows(h, j + 1 + t); n2_h[q] = nbj; k2_h[q] = P.rk[id];
        a2_h[q] = P.uoff[id];
        b2_h[q] = (int64_t)t * nb * nb;
        c2_h[q] = (int64_t)nbj + (int64_t)t * nb;
        mmax = std::max(mmax, m2_h[q]);
        cf += 2.0 * m2_h[q] * nbj * P.rk[id];
        ++q;
      }
      im_push(h, m2_h, m_d, 3 * (int64_t)cnt);
      lm_push(h, a2_h, a_d, 3 * (int64_t)cnt);
      // dC_ij -= U_ij P_t^T: inner dimension a rank, streamed over the column
      GemmBatch cb{};
      cb.count = cnt; cb.m_of = m_d; cb.n_of = n_d; cb.k_of = k_d; cb.a_off = a_d; cb.b_off = b_d; cb.c_off = c_d;
      rest_wait();
      if (kmax <= kThinMaxK) {
        HIPCHK(launch_thin_gemm(h->arena, nb, h->Ptmp, nb, cold, h->n, cb, mmax, kmax, nbj, h->s, -1.0, 1.0, true));
      } else {
        GemmSeg cs{};
        cs.A = op_contig(h->arena, nb, 0, 0);
        cs.B = op_contig(h->Ptmp, nb, 0, 0);
        cs.K = kmax;
        gemm(h, mmax, nbj, 1, &cs, cold, h->n, epi_linear(-1.0, 1.0), &cb);
      }
    }
    prof_add(h, TLR_K_LOWRANK, e_c, cf, 0.0);
  };
  auto tangent_job = [&](int j) {
    const int T = nt - j - 1;
    return ColumnJob{tbuf(j) + tile_rows(h, j), j + 1, T, j, &G, predict_ranks(h, G, j, T),
                     h->dinv_off + (int64_t)j * nb * nb, 0};
  };
  // compress, then V <- L_jj^{-1} V; with the look-ahead the diagonal step
  // of the newest primal column runs beside the compression (only the
  // triangular solves need it), so the main stream waits for it in between
  auto finish = [&](std::vector<ColumnJob>& jobs, bool wait_diag, std::function<void()> during0 = nullptr,
                    std::function<void()> during1 = nullptr) {
    std::function<void()> during[2] = {std::move(during0), std::move(during1)};
    compress_columns(h, jobs, during);
    for (auto& f : during)
      if (f) f();
    if (wait_diag) HIPCHK(hipStreamWaitEvent(h->s_main, h->ev_diag, 0));
    dbg_mark(h, 9, h->s_main);
    dbg_host(h, 2);
    for (const ColumnJob& jb : jobs)
      if (jb.T > 0) lowrank_trsm(h, jb.col, jb.i_first, jb.T, h->Vtmp + (int64_t)jb.g0 * h->vslot, *jb.F);
    dbg_host(h, 3);
  };

  if (!side) {
    // one stream: each step updates, factors and compresses its columns in turn
    primal_update(0, 0, 0, true);
    primal_diag(0);
    {
      std::vector<ColumnJob> jobs{primal_job(0)};
      finish(jobs, false);
    }
    for (int j = 0; j < nt; ++j) {
      std::vector<ColumnJob> jobs;
      if (j + 1 < nt) {
        primal_update(j + 1, 0, j + 1, true);
        primal_diag(j + 1);
        jobs.push_back(primal_job(j + 1));
      }
      if (tangent) {
        tangent_update(j, 0, j, true);
        tangent_rest(j);
        jobs.push_back(tangent_job(j));
      }
      finish(jobs, false);
    }
  } else {
    // Two streams, lockstep with look-ahead.  Step j compresses primal column
    // j + 1 and tangent column j together (main stream).  Everything of those
    // columns that does not depend on step j - 1's compressions (generation
    // and the terms of columns up to j - 1 for the primal, up to j - 2 for the
    // tangent: "pre") runs on the side stream while step j - 1 compresses;
    // afterwards the last term, the diagonal steps and the tangent's
    // correction ("post") complete them, the primal on the main stream and
    // the tangent on the side stream; the last terms beyond the diagonal
    // tiles (and the tangent's correction) are folded into the compression.
    auto pre = [&](int j) {   // side stream: pre parts of step j
      SideStream ss(h);
      if (j + 1 < nt) primal_update(j + 1, 0, j, true);
      tangent_update(j, 0, j - 1, true);
      HIPCHK(hipEventRecord(h->ev_pre, h->s));
      dbg_mark(h, 12, h->s);
    };
    primal_update(0, 0, 0, true);
    primal_diag(0);
    {
      std::vector<ColumnJob> jobs{primal_job(0)};
      finish(jobs, false);
    }
    HIPCHK(hipEventRecord(h->ev_fin, h->s_main));
    {
      SideStream ss(h);
      HIPCHK(hipStreamWaitEvent(h->s, h->ev_fin, 0));
    }
    pre(0);
    for (int j = 0; j < nt; ++j) {
      // main: the rest of primal column j + 1 waits for its pre part
      HIPCHK(hipStreamWaitEvent(h->s_main, h->ev_pre, 0));
      h->dbg_step = j;
      dbg_mark(h, 0, h->s_main);
      dbg_host(h, 4);
      // Issued first: the primal column's rest and then its sketch are the
      // longer chain to the next compression; the host issues launches about
      // as fast as the GPU runs these short kernels.
      // The last term of primal column j + 1 updates only its diagonal tile
      // here; the tiles below take it inside their compression (fold).
      FoldOut pfold, tfold;
      pfold.wdst = h->Wf;
      pfold.wld = h->wf_ld;
      pfold.wcols = h->wf_pcols;
      if (j + 1 < nt) {
        primal_update(j + 1, j, j + 1, false, &pfold);
        HIPCHK(hipEventRecord(h->ev_post, h->s_main));
        dbg_mark(h, 1, h->s_main);
      }
      {
        // side: the rest of tangent column j, after step j - 1's compressions
        SideStream ss(h);
        HIPCHK(hipStreamWaitEvent(h->s, h->ev_fin, 0));
        dbg_mark(h, 2, h->s);
        // the tangent's last term beyond its diagonal tile and its correction
        // folded into the compression when they fit (tfold.K > 0); else the
        // rows below on the diagonal-step stream (idle here), beside the
        // tangent of the diagonal step, and the correction here
        if (!tangent_fold_setup(j, tfold)) tfold = FoldOut{};
        tangent_update(j, j - 1, j, false, h->s_diag, tfold.wdst ? &tfold : nullptr);
        dbg_mark(h, 14, h->s);
        tangent_rest(j, &tfold);
        rest_wait();
        HIPCHK(hipEventRecord(h->ev_join, h->s));
        dbg_mark(h, 3, h->s);
        dbg_host(h, 5);
      }
      // the diagonal step of primal column j + 1 on its own stream, behind the
      // tangent's rows there: only the triangular solves after the
      // compression need it, and issued here it runs beside the compression
      if (j + 1 < nt) {
        DiagStream ds(h);
        HIPCHK(hipStreamWaitEvent(h->s, h->ev_post, 0));
        primal_diag(j + 1);
        HIPCHK(hipEventRecord(h->ev_diag, h->s));
        dbg_mark(h, 11, h->s);
        dbg_host(h, 6);
      }
      // each column is sketched as soon as it is complete: the primal one on
      // the main stream, the tangent one on the side stream after its chain
      std::vector<ColumnJob> jobs;
      if (j + 1 < nt) {
        jobs.push_back(primal_job(j + 1));
        jobs.back().fold = pfold;
      }
      jobs.push_back(tangent_job(j));
      jobs.back().wait = h->ev_join;
      jobs.back().fold = tfold;
      jobs.back().sketch_stream = h->s_side;
      // The compressions of step j are issued first; the host issues the pre
      // parts of step j + 1 (side stream) in its first wait, for the range
      // ranks.
      finish(jobs, j + 1 < nt, [&]() {
        if (j + 1 < nt) pre(j + 1);
      });
      HIPCHK(hipEventRecord(h->ev_fin, h->s_main));
      dbg_mark(h, 10, h->s_main);
    }
  }
  family_upload(h, P);
  sync(h);
  if (h->debug) {
    std::fprintf(stderr,
                 "[tlr] host ms: issue in wait 1 %.1f, wait 1 %.1f, issue in wait 2 %.1f, wait 2 %.1f, "
                 "wait 2 to upload %.1f, upload %.1f, upload to last launch %.1f; staging syncs %d (main %d)\n",
                 h->host_ms[0], h->host_ms[1], h->host_ms[2], h->host_ms[3], h->host_ms[4], h->host_ms[5],
                 h->host_ms[6], h->dbg_meta_syncs, h->dbg_meta_syncs_main);
    h->dbg_meta_syncs = h->dbg_meta_syncs_main = 0;
    for (double& v : h->host_ms) v = 0.0;
    dbg_report(h);
  }
  h->dbg_step = -1;
  P.done_kind = 1;
  if (tangent) G.done_kind = 1;
}

// log|Sigma~| and y = L^{-1} z (into vec[1]); returns (logdet, quad)
// largest rank of the tiles below the diagonal in column j (col) or left of
// it in row j (!col), for the low-rank apply launches
int lr_kmax(const tlr_handle_s* h, int j, bool col) {
  const Family& F = h->fam[0];
  int km = 0;
  if (col)
    for (int i = j + 1; i < h->nt; ++i) km = std::max(km, F.rk[tid_of(h, i, j)]);
  else
    for (int k = 0; k < j; ++k) km = std::max(km, F.rk[tid_of(h, j, k)]);
  return km;
}

void solve_forward(tlr_handle_s* h, const double* z, double* logdet, double* quad) {
  const int nt = h->nt, nb = h->nb;
  const int64_t n = h->n;
  double* w = h->vec;
  double* ys = h->vec + n;
  HIPCHK(launch_copy_block(z, n, w, n, n, 1, h->s));
  for (int j = 0; j < nt; ++j) {
    const int nbj = tile_rows(h, j);
    const int64_t r0 = (int64_t)j * nb;
    HIPCHK(launch_gemv_n(dinv_tile(h, j), nb, nbj, nbj, w + r0, 1.0, 0.0, ys + r0, h->s));
    if (j + 1 < nt) {
      if (h->dense) {
        const int64_t ldp = n - r0;
        HIPCHK(launch_gemv_n(panel(h, h->Lp, j) + nbj, ldp, n - r0 - nbj, nbj, ys + r0, -1.0, 1.0, w + r0 + nbj,
                             h->s));
      } else {
        LowRankApply a{};
        a.arena = h->arena; a.uoff = h->fam[0].uoff_d; a.voff = h->fam[0].voff_d; a.ranks = h->fam[0].rk_d;
        a.n = n; a.nb = nb; a.nt = nt; a.fixed = j; a.forward = 1; a.v = ys; a.out = w; a.scale = -1.0;
        a.tws = h->lrtws;
        HIPCHK(launch_lowrank_apply(a, nt - j - 1, h->s, lr_kmax(h, j, true)));
      }
    }
  }
  HIPCHK(launch_dot(ys, ys, n, h->scal + 2 * nt, h->s));
  HIPCHK(hipMemcpyAsync(h->h_scal, h->scal, (2 * nt + 1) * sizeof(double), hipMemcpyDeviceToHost, h->s));
  sync(h);
  double ld = 0.0;
  for (int j = 0; j < nt; ++j) ld += h->h_scal[j];
  *logdet = 2.0 * ld;
  *quad = h->h_scal[2 * nt];
}

// a = L^{-T} y with y = vec[1] (from solve_forward); result in vec[2]
void solve_backward(tlr_handle_s* h) {
  const int nt = h->nt, nb = h->nb;
  const int64_t n = h->n;
  double* ys = h->vec + n;
  double* al = h->vec + 2 * n;
  double* r = h->vec + 3 * n;
  HIPCHK(launch_copy_block(ys, n, r, n, n, 1, h->s));
  for (int i = nt - 1; i >= 0; --i) {
    const int nbi = tile_rows(h, i);
    const int64_t r0 = (int64_t)i * nb;
    if (h->dense && i + 1 < nt) {
      const int64_t ldp = n - r0;
      HIPCHK(launch_gemv_t(panel(h, h->Lp, i) + nbi, ldp, n - r0 - nbi, nbi, al + r0 + nbi, -1.0, 1.0, r + r0, h->s));
    }
    HIPCHK(launch_gemv_t(dinv_tile(h, i), nb, nbi, nbi, r + r0, 1.0, 0.0, al + r0, h->s));
    if (!h->dense && i > 0) {
      LowRankApply a{};
      a.arena = h->arena; a.uoff = h->fam[0].uoff_d; a.voff = h->fam[0].voff_d; a.ranks = h->fam[0].rk_d;
      a.n = n; a.nb = nb; a.nt = nt; a.fixed = i; a.forward = 0; a.v = al; a.out = r; a.scale = -1.0;
      a.tws = h->lrtws;
      HIPCHK(launch_lowrank_apply(a, i, h->s, lr_kmax(h, i, false)));
    }
  }
}

tlr_status check_info(tlr_handle_s* h, int64_t* info) {
  HIPCHK(hipMemcpyAsync(h->h_info, h->info_d, sizeof(unsigned long long), hipMemcpyDeviceToHost, h->s));
  sync(h);
  const unsigned long long v = *h->h_info;
  if (v != ~0ull) {
    if (info) *info = (int64_t)v;
    return TLR_ENOTSPD;
  }
  if (info) *info = 0;
  return TLR_OK;
}

// Factorisation with its definiteness check.  With FP32 update products the
// rounding of the densely accumulated updates (about 1e-7 of their size, full
// rank) can push a pivot of an ill-conditioned Sigma below zero although
// Sigma is positive definite: such a factor is computed again with FP64
// products, and the info counters record it.  The handle keeps FP64 products
// from then on: its later calls (nearby theta of the same field) would most
// likely fail the same way and pay for two factorisations.
// Automatic tile storage (opts.arena_bytes == 0) that ran out: twice the
// capacity, and the caller starts the pass again.
void arena_grow(tlr_handle_s* h) {
  h->s = h->s_main;   // an interrupted pass may have left a side stream current
  h->tile_overflow = false;
  ++h->arena_grows;
  arena_alloc(h, 2 * h->tile_cap);
}

tlr_status factor_checked(tlr_handle_s* h, bool tangent, int64_t* info) {
  const bool f32 = h->o.prec == TLR_PREC_FP32_UPDATES && h->info.fp64_retries == 0;
  h->upd_tag = f32 ? 2 : 1;
  h->info.prec_used = f32 ? TLR_PREC_FP32_UPDATES : TLR_PREC_FP64;
  for (;;) {
    tlr_status st;
    h->splitk_count = 0;
    try {
      if (h->dense) factor_dense(h, tangent); else factor_tlr(h, tangent);
      st = check_info(h, info);
      h->info.splitk_launches = h->splitk_count;
    } catch (const Fail& f) {
      if (f.st == TLR_ENOMEM && h->tile_overflow && h->tile_auto) {
        arena_grow(h);
        continue;
      }
      if (f.st != TLR_ENOTSPD) throw;
      st = check_info(h, info);
    }
    if (st != TLR_ENOTSPD || h->upd_tag != 2) return st;
    drop_history(h);
    h->upd_tag = 1;
    h->info.prec_used = TLR_PREC_FP64;
    ++h->info.fp64_retries;
  }
}

void rank_stats(tlr_handle_s* h) {
  int64_t sum = 0;
  int mx = 0, nd = 0;
  const Family& F = h->fam[0];
  for (int i = 0; i < h->nt; ++i)
    for (int j = 0; j < i; ++j) {
      const size_t id = (size_t)i * h->nt + j;
      if (F.isdense[id]) {
        ++nd;
        continue;
      }
      sum += F.rk[id];
      mx = std::max(mx, F.rk[id]);
    }
  h->info.rank_sum = sum;
  h->info.rank_max = mx;
  h->info.dense_tiles = nd;
  h->info.tile_bytes_used = h->tile_used * (int64_t)sizeof(double);
  h->info.tile_bytes_cap = h->tile_cap * (int64_t)sizeof(double);
  h->info.arena_grows = h->arena_grows;
  h->info.qr_tiles_reg = h->qr_class[0];
  h->info.qr_tiles_lds = h->qr_class[1];
  h->info.qr_tiles_global = h->qr_class[2];
  h->info.device_bytes = h->bytes;
}


void free_all(tlr_handle_s* h) {
  if (h->s_main) (void)hipStreamSynchronize(h->s_main);
  for (hipStream_t* st : {&h->s_side, &h->s_diag}) {
    if (!*st) continue;
    (void)hipStreamSynchronize(*st);
    (void)hipStreamDestroy(*st);
    *st = nullptr;
  }
  for (hipEvent_t* e : {&h->ev_fork, &h->ev_join, &h->ev_px, &h->ev_py, &h->ev_pre, &h->ev_fin, &h->ev_post,
                        &h->ev_diag, &h->ev_rw, &h->ev_rest}) {
    if (*e) (void)hipEventDestroy(*e);
    *e = nullptr;
  }
  for (void* p : h->dev_allocs) (void)hipFree(p);
  if (h->arena) (void)hipFree(h->arena);
  h->arena = nullptr;
  for (void* p : h->host_allocs) (void)hipHostFree(p);
  for (hipEvent_t& e : h->ev)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t& e : h->evpool) (void)hipEventDestroy(e);
  h->evpool.clear();
  for (hipEvent_t& e : h->dbg_ev)
    if (e) (void)hipEventDestroy(e);
  h->dbg_ev.clear();
  h->dev_allocs.clear();
  h->host_allocs.clear();
}

float elapsed(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) {
    (void)hipGetLastError();
    return 0.f;
  }
  return ms;
}

// tlr_compress: every strictly-lower tile of Sigma compressed (no factorisation)
void compress_sigma(tlr_handle_s* h) {
  {
    prof_reset_pool(h);
    const int nt = h->nt, nb = h->nb;
    Family& F = h->fam[0];
    family_reset(h, F, 2);
    h->tile_used = 0;
    h->tile_overflow = false;
    reset_info(h);
    sync(h);
    meta_reset(h);
    h->state = 0;
    for (int j = 0; j < nt; ++j) {
      const int nbj = tile_rows(h, j);
      HIPCHK(launch_matern_block(h->mp, h->x, h->y, (int64_t)j * nb, nbj, (int64_t)j * nb, nbj, diag_tile(h, j), nb,
                                 false, h->s));
      const int T = nt - j - 1;
      if (T <= 0) continue;
      const int64_t rows = h->n - (int64_t)(j + 1) * nb;
      HIPCHK(launch_matern_block(h->mp, h->x, h->y, (int64_t)(j + 1) * nb, rows, (int64_t)j * nb, nbj, h->col,
                                 h->n, false, h->s));
      std::vector<ColumnJob> jobs{ColumnJob{h->col, j + 1, T, j, &F, predict_ranks(h, F, j, T), h->ident_off, 0}};
      compress_columns(h, jobs);
      // low-rank V slots <- V~ (no TRSM: this is Sigma itself)
      int cnt = 0;
      for (int t = 0; t < T; ++t) {
        const size_t id = tid_of(h, j + 1 + t, j);
        if (!F.isdense[id] && F.rk[id] > 0) ++cnt;
      }
      if (cnt == 0) continue;
      meta_reserve(h, 2 * (int64_t)cnt, 2 * (int64_t)cnt);
      int *m_d, *k_d;
      int* m_h = im_take(h, cnt, &m_d);
      int* k_h = im_take(h, cnt, &k_d);
      int64_t *so_d, *do_d;
      int64_t* so_h = lm_take(h, cnt, &so_d);
      int64_t* do_h = lm_take(h, cnt, &do_d);
      int64_t maxe = 0;
      int q = 0;
      for (int t = 0; t < T; ++t) {
        const size_t id = tid_of(h, j + 1 + t, j);
        if (F.isdense[id] || F.rk[id] <= 0) continue;
        m_h[q] = nbj;
        k_h[q] = F.rk[id];
        so_h[q] = (int64_t)t * h->vslot;
        do_h[q] = F.voff[id];
        maxe = std::max<int64_t>(maxe, (int64_t)nbj * k_h[q]);
        ++q;
      }
      im_push(h, m_h, m_d, 2 * (int64_t)cnt);
      lm_push(h, so_h, so_d, 2 * (int64_t)cnt);
      HIPCHK(launch_batched_copy(h->Vtmp, nb, so_d, h->arena, nb, do_d, m_d, k_d, maxe, cnt, h->s));
    }
    family_upload(h, F);
    sync(h);
    F.done_kind = 2;
    rank_stats(h);
    h->state = 1;
  }
}

// tlr_compress with TLR_FLAG_ACA: every strictly-lower tile of Sigma by
// adaptive cross approximation fused with its generation (aca.hip), column
// by column; U and V go to the tile storage at the rank ACA stopped at.  The
// stop is two consecutive terms with ||u|| ||v|| <= tol / 10.  A tile that
// needs more than maxrank steps is generated densely (V = identity), or is a
// TLR_ERANK failure with TLR_FLAG_STRICT_RANK.
void compress_sigma_aca(tlr_handle_s* h) {
  prof_reset_pool(h);
  const int nt = h->nt, nb = h->nb;
  Family& F = h->fam[0];
  family_reset(h, F, 2);
  h->tile_used = 0;
  h->tile_overflow = false;
  reset_info(h);
  sync(h);
  meta_reset(h);
  h->state = 0;
  const int kmax = h->maxrank;
  const double tau = 0.1 * h->o.tol;
  double cflops = 0.0;
  for (int j = 0; j < nt; ++j) {
    const int nbj = tile_rows(h, j);
    HIPCHK(launch_matern_block(h->mp, h->x, h->y, (int64_t)j * nb, nbj, (int64_t)j * nb, nbj, diag_tile(h, j), nb,
                               false, h->s));
    const int T = nt - j - 1;
    if (T <= 0) continue;
    const size_t e_c = prof_mark(h);
    for (int t = 0; t < T; ++t) {
      AcaTask& a = h->aca_h[t];
      a.r0 = (int64_t)(j + 1 + t) * nb;
      a.c0 = (int64_t)j * nb;
      a.m = tile_rows(h, j + 1 + t);
      a.n = nbj;
      a.U = h->Ybuf + (int64_t)t * nb * h->smax;
      a.V = h->Q1 + (int64_t)t * nb * h->smax;
      a.ld = nb;
      a.rank = h->qr_d + t;
    }
    HIPCHK(hipMemcpyAsync(h->aca_d, h->aca_h, T * sizeof(AcaTask), hipMemcpyHostToDevice, h->s));
    HIPCHK(launch_aca(h->mp, h->x, h->y, h->aca_d, T, kmax, tau, h->s));
    HIPCHK(hipMemcpyAsync(h->qr_h, h->qr_d, T * sizeof(int), hipMemcpyDeviceToHost, h->s));
    HIPCHK(hipStreamSynchronize(h->s));
    meta_reset(h);
    int nlr = 0;
    for (int t = 0; t < T; ++t) {
      const int i = j + 1 + t;
      const size_t id = tid_of(h, i, j);
      const int k = h->qr_h[t];
      const int m = tile_rows(h, i);
      cflops += 2.0 * k * (double)k * (m + nbj);
      if (k > kmax) {
        if (h->strict) {
          h->bad_i = i;
          h->bad_j = j;
          throw Fail{TLR_ERANK};
        }
        F.isdense[id] = 1;
        F.rk[id] = nbj;
        F.uoff[id] = tile_take(h, (int64_t)nb * nbj);
        F.voff[id] = h->ident_off;
        HIPCHK(launch_matern_block(h->mp, h->x, h->y, (int64_t)i * nb, m, (int64_t)j * nb, nbj,
                                   h->arena + F.uoff[id], nb, false, h->s));
      } else {
        F.rk[id] = k;
        F.uoff[id] = k > 0 ? tile_take(h, (int64_t)nb * k) : 0;
        F.voff[id] = k > 0 ? tile_take(h, (int64_t)nb * k) : 0;
        if (k > 0) ++nlr;
      }
    }
    if (nlr > 0) {
      // U (m x k) and V (nbj x k) from the ACA scratch to the tile storage
      meta_reserve(h, 4 * (int64_t)nlr, 4 * (int64_t)nlr);
      int *m_d, *k_d;
      int* m_h = im_take(h, 2 * nlr, &m_d);
      int* k_h = im_take(h, 2 * nlr, &k_d);
      int64_t *so_d, *do_d;
      int64_t* so_h = lm_take(h, 2 * nlr, &so_d);
      int64_t* do_h = lm_take(h, 2 * nlr, &do_d);
      int q = 0;
      int64_t maxe = 0;
      for (int t = 0; t < T; ++t) {
        const size_t id = tid_of(h, j + 1 + t, j);
        if (F.isdense[id] || F.rk[id] <= 0) continue;
        const int k = F.rk[id];
        m_h[q] = tile_rows(h, j + 1 + t); k_h[q] = k;
        m_h[nlr + q] = nbj; k_h[nlr + q] = k;
        so_h[q] = so_h[nlr + q] = (int64_t)t * nb * h->smax;   // same block of the U and the V scratch
        do_h[q] = F.uoff[id];
        do_h[nlr + q] = F.voff[id];
        maxe = std::max<int64_t>(maxe, (int64_t)nb * k);
        ++q;
      }
      im_push(h, m_h, m_d, 2 * (int64_t)nlr);
      im_push(h, k_h, k_d, 2 * (int64_t)nlr);
      lm_push(h, so_h, so_d, 2 * (int64_t)nlr);
      lm_push(h, do_h, do_d, 2 * (int64_t)nlr);
      HIPCHK(launch_batched_copy(h->Ybuf, nb, so_d, h->arena, nb, do_d, m_d, k_d, maxe, nlr, h->s));
      HIPCHK(launch_batched_copy(h->Q1, nb, so_d + nlr, h->arena, nb, do_d + nlr, m_d + nlr, k_d + nlr, maxe, nlr,
                                 h->s));
    }
    prof_add(h, TLR_K_COMPRESS, e_c, 0.0, 0.0);
  }
  family_upload(h, F);
  sync(h);
  F.done_kind = 2;
  rank_stats(h);
  h->state = 1;
  (void)cflops;
}

}  // namespace tlri
