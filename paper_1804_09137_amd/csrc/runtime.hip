// Host runtime of the factorisation: error reporting, the pinned staging of
// launch metadata, the stream roles and the rank read-backs, the per-class
// timing of launch groups, the GEMM dispatch (operands, epilogues, split-K
// and tile choice) and the tile bookkeeping of a TLR family.
#include "factor.h"

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
// When the new size cannot be had, the previous size is taken again (so that
// the handle keeps storage for its next pass) and TLR_ENOMEM is reported.
void arena_alloc(tlr_handle_s* h, int64_t cap) {
  const int64_t nb = h->nb, nt = h->nt;
  const int64_t prev_cap = h->arena ? h->tile_cap : -1;
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
    if (prev_cap >= 0 && prev_cap < h->tile_cap) {
      try {
        arena_alloc(h, prev_cap);
      } catch (const Fail&) {
        // left without an arena: arena_ensure() retries before the next pass
      }
    }
    throw Fail{TLR_ENOMEM};
  }
  h->arena = (double*)p;
  h->bytes += h->arena_len * (int64_t)sizeof(double);
  h->Dinv = h->arena + h->dinv_off;
  h->tile_used = 0;
  HIPCHK(launch_fill(h->arena + h->ident_off, nb, nb, nb, 0.0, h->s));
  HIPCHK(launch_identity(h->arena + h->ident_off, nb, nb, h->s));
}

// A TLR handle whose arena could not be reallocated gets it back (at the
// capacity last asked for) before a pass uses it, or the pass fails with
// TLR_ENOMEM.
void arena_ensure(tlr_handle_s* h) {
  if (!h->dense && !h->arena) arena_alloc(h, h->tile_cap);
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


}  // namespace tlri
