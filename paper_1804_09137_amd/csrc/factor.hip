// Factorisation drivers: the dense and tile low-rank Cholesky of Sigma(theta)
// (with their tangents for the gradient), the solves, the compression of
// Sigma alone and the handle's memory.  The host runtime they run on is in
// runtime.hip, the compression of tile columns in compress_cols.hip and the
// column update in column_update.hip.
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
#include "factor.h"

#include <array>
#include <atomic>
#include <system_error>
#include <thread>

using namespace tlrk;

namespace tlri {

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
  arena_ensure(h);
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
