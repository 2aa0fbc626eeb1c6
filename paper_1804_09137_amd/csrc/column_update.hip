// ---------------------------------------------------------------------------
// W-build and column GEMM of the TLR factorisation:
// C(i, j) = Gen(i, j) - sum_terms sum_k L1(i,k) L2(j,k)^T, i in [j, nt),
// L1(i,k) L2(j,k)^T = U1_ik (V1_ik^T V2_jk) U2_jk^T, written to out (row
// offset (i - j) nb, ld n).  Gen is Sigma (primal) or dSigma/dbeta (tangent).
// ---------------------------------------------------------------------------
#include "factor.h"

#include <array>
#include <atomic>
#include <system_error>
#include <thread>

using namespace tlrk;

namespace tlri {

// Column j of Sigma (or dSigma/dbeta, by epi_kind) minus the terms k in
// [kb, ke) of the left-looking sum: gen = true writes the generated block
// first, gen = false subtracts from what out already holds.  A column can so
// take most of its terms while an earlier column is still being compressed,
// and the rest afterwards.
// rest_on: the rows below the diagonal tile are updated on that stream
// (ev_rest recorded there, rest_pending set): the diagonal tile is ready
// sooner for what follows on this stream.
void tlr_column_update(tlr_handle_s* h, int j, int nterms, const LRTerm* terms, double* out, int epi_kind, int kb,
                       int ke, bool gen, FoldOut* fold, hipStream_t rest_on) {
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

}  // namespace tlri
