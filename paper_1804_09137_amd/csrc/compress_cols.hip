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
#include "factor.h"

#include <array>
#include <atomic>
#include <system_error>
#include <thread>

using namespace tlrk;

namespace tlri {

// during[0], during[1]: host work to do while the compression's launches run,
// each called once: the first before the wait for the range ranks, the second
// before the wait for the truncation ranks (the caller calls what is left when
// no tile needed that wait).  Each host wait then costs the main stream no
// launch time: the launches that follow it are issued as soon as it ends.
void compress_columns(tlr_handle_s* h, std::vector<ColumnJob>& jobs, std::function<void()>* during) {
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

}  // namespace tlri
