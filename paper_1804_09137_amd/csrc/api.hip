// C-ABI entry points (include/tlr.h).  Each call validates its arguments,
// then runs the factorisation drivers under guarded(), which turns internal
// failures into status codes.
#include "handle.h"

#include <atomic>
#include <system_error>
#include <thread>

using namespace tlrk;
using namespace tlri;

// ===========================================================================
// C-ABI
// ===========================================================================
extern "C" {

const char* tlr_last_error(void) { return g_last_error; }

tlr_status tlr_create(tlr_handle_t* out, const tlr_opts* o, void* stream) {
  if (!out || !o) return TLR_EINVAL;
  *out = nullptr;
  if (o->n < 1 || o->nb < 32 || o->nb > kQrMaxRows || o->nb % 16 != 0) return TLR_EINVAL;
  if (o->mode != TLR_MODE_TLR && o->mode != TLR_MODE_DENSE) return TLR_EINVAL;
  if (o->prec != TLR_PREC_FP64 && o->prec != TLR_PREC_FP32_UPDATES) return TLR_EINVAL;
  if (o->mode == TLR_MODE_TLR && !(o->tol > 0.0 && std::isfinite(o->tol))) return TLR_EINVAL;
  if (o->prec == TLR_PREC_FP32_UPDATES && o->mode != TLR_MODE_TLR) return TLR_EINVAL;
  if (o->arena_bytes < 0) return TLR_EINVAL;
  if (o->metric != TLR_METRIC_EUCLID && o->metric != TLR_METRIC_GREAT_CIRCLE) return TLR_EINVAL;
  if (!(o->sphere_radius >= 0.0 && std::isfinite(o->sphere_radius))) return TLR_EINVAL;
  tlr_handle_s* h = new (std::nothrow) tlr_handle_s();
  if (!h) return TLR_ENOMEM;
  tlr_status st = guarded(h, [&]() -> tlr_status {
    h->o = *o;
    h->s = h->s_main = (hipStream_t)stream;
    HIPCHK(hipGetDevice(&h->device));
    h->n = o->n;
    h->nb = o->nb;
    h->nt = (int)((o->n + o->nb - 1) / o->nb);
    h->dense = (o->mode == TLR_MODE_DENSE);
    h->grad = o->want_grad != 0;
    int mr = o->maxrank > 0 ? o->maxrank : o->nb / 4;
    mr = std::min(mr, o->nb);
    mr = std::min(mr, kQrMaxCols - 96);
    h->maxrank = mr;
    h->strict = (o->flags & TLR_FLAG_STRICT_RANK) != 0;
    h->pivoted_trunc = (o->flags & TLR_FLAG_PIVOTED_TRUNC) != 0;
    // TLR gradient handles run the tangent chain and the diagonal steps on
    // streams of their own unless asked for one stream
    h->multi = h->grad && !h->dense && !(o->flags & TLR_FLAG_SINGLE_STREAM);
    const int mslot = mr;
    // sketch width cap: a tile whose range finder needs more columns than
    // this is (unless strict) kept dense
    h->smax = (int)std::min<int64_t>(kQrMaxCols, pad16(mr + mr / 2 + 48));
    h->debug = std::getenv("TLR_DEBUG") != nullptr;
    h->vslot = (int64_t)o->nb * (mslot + 1);
    h->ntiles = (int64_t)h->nt * (h->nt - 1) / 2;
    const int64_t n = h->n, nb = h->nb, nt = h->nt;
    const int nterms = h->grad ? 2 : 1;
    h->d_tab = dalloc<double>(h, kTabSize);
    h->h_tab.assign(kTabSize, 0.0);
    if (h->dense) h->Dinv = dalloc<double>(h, nt * nb * nb);
    // one allocation: compressions address the tiles of every column buffer from h->colbase
    h->colbase = dalloc<double>(h, n * nb * (h->multi ? 4 : (h->grad ? 2 : 1)));
    h->col = h->colbase;
    if (h->grad) h->cold = h->colbase + n * nb;
    if (h->multi) {
      h->col2 = h->colbase + 2 * n * nb;
      h->cold2 = h->colbase + 3 * n * nb;
    }
    h->tw = dalloc<double>(h, 64 * nb + 3 * nb * nb);
    h->vec = dalloc<double>(h, 4 * n);
    h->scal = dalloc<double>(h, 4 * nt + 16);
    h->h_scal = halloc<double>(h, 4 * nt + 16);
    h->info_d = dalloc<unsigned long long>(h, 1);
    h->h_info = halloc_coherent<unsigned long long>(h, 1, &h->h_info_d);
    h->pub_seq_h = halloc_coherent<unsigned>(h, 1, &h->pub_seq_d);
    *h->pub_seq_h = 0;
    h->sk_cap = std::min<int64_t>(16ll << 20, 32 * std::max<int64_t>(n, 1024) * nb);
    h->skw = dalloc<double>(h, h->sk_cap);
    if (h->dense) {
      h->Lp = dalloc<double>(h, panels_size(n, nb));
      if (h->grad) {
        h->Ldp = dalloc<double>(h, panels_size(n, nb));
        // metadata of the tangent's batched diagonal products
        h->im_cap = 1 << 16;
        h->lm_cap = 1 << 15;
        h->im_d = dalloc<int>(h, h->im_cap);
        h->im_h = halloc<int>(h, h->im_cap);
        h->lm_d = dalloc<int64_t>(h, h->lm_cap);
        h->lm_h = halloc<int64_t>(h, h->lm_cap);
      }
    } else {
      h->D = dalloc<double>(h, nt * nb * nb);
      if (h->grad) h->Dd = dalloc<double>(h, nt * nb * nb);
      h->lrtws = dalloc<double>(h, nt * (int64_t)kLrMaxRank);
      // arena: identity, Dinv tiles, tile storage.  Explicit arena_bytes:
      // that much tile storage, fixed.  Otherwise room for every tile of
      // every family at rank max(12, maxrank / 16) plus one dense tile per
      // tile column, grown (doubled) when a factorisation needs more.
      const int nfam = h->grad ? 2 : 1;
      int64_t cap;
      if (o->arena_bytes > 0) {
        h->tile_auto = false;
        cap = o->arena_bytes / (int64_t)sizeof(double);
      } else {
        const int64_t rg = std::max<int64_t>(12, mr / 16);
        cap = nfam * (h->ntiles * 2 * nb * pad16(rg) + nt * nb * nb);
        // TLR_ARENA_START (doubles) lowers the first automatic capacity, so
        // that tests reach the doubling (at least kAlign: a capacity that
        // rounds down to 0 would double to 0 forever)
        if (const char* as = std::getenv("TLR_ARENA_START"))
          cap = std::min<int64_t>(cap, std::max<int64_t>(kAlign, std::atoll(as)));
      }
      for (int f = 0; f < 2; ++f) {
        Family& F = h->fam[f];
        F.rk.assign((size_t)nt * nt, 0);
        F.r1.assign((size_t)nt * nt, 0);
        F.r1_prev.assign((size_t)nt * nt, 0);
        F.rk_prev.assign((size_t)nt * nt, 0);
        F.uoff.assign((size_t)nt * nt, 0);
        F.voff.assign((size_t)nt * nt, 0);
        F.isdense.assign((size_t)nt * nt, 0);
        F.dense_meas.assign((size_t)nt * nt, 0);
        F.dense_meas_prev.assign((size_t)nt * nt, 0);
        F.rk_d = dalloc<int>(h, nt * nt);
        F.uoff_d = dalloc<int64_t>(h, nt * nt);
        F.voff_d = dalloc<int64_t>(h, nt * nt);
      }
      arena_alloc(h, cap);
      if (h->grad) {
        h->ptmp_cap = nt * nb * nb;
        h->Ptmp = dalloc<double>(h, h->ptmp_cap);
      }
      h->omega = dalloc<double>(h, nb * h->smax);
      h->gcap = (int)(h->grad ? 2 * nt : nt);   // tiles compressed together: two columns with the tangent
      const int64_t gc = h->gcap;
      h->Ybuf = dalloc<double>(h, gc * nb * h->smax);
      h->Q1 = dalloc<double>(h, gc * nb * h->smax);
      h->Bt = dalloc<double>(h, gc * nb * h->smax);
      h->Vtmp = dalloc<double>(h, gc * h->vslot);
      h->Zb = dalloc<double>(h, gc * h->smax * (mslot + 1));
      // the right factors of one row of tiles, side by side: up to rmax
      // columns (a dense tile counts nb).  Every tile of a row dense when
      // that takes at most 64 Mi doubles; beyond, ranks averaging maxrank / 2
      // plus eight dense tiles per row, and a row needing more fails with
      // TLR_ENOMEM
      int64_t rmax = nterms * nt * nb;
      if (nb * rmax > (64ll << 20)) rmax = std::min<int64_t>(rmax, nterms * (nt * std::max(mr / 2, 16) + 8 * nb));
      h->urow_cap = nb * rmax;
      h->Urow = dalloc<double>(h, h->urow_cap);
      // W (rows below the diagonal x row rank sum) and the X = V^T V blocks
      // are taken in chunks of tile rows that fit these capacities
      int64_t wworst = 0, xworst = 0;
      for (int64_t j = 0; j < nt; ++j) {
        wworst = std::max(wworst, (nt - j) * nb * nterms * j * nb);
        xworst = std::max(xworst, (nt - j) * nterms * j * nb * nb);
      }
      h->w_cap = std::max<int64_t>(std::min<int64_t>(wworst, 160ll << 20), nb * rmax);
      h->x_cap = std::max<int64_t>(std::min<int64_t>(xworst, 64ll << 20), nb * rmax);
      h->Wb = dalloc<double>(h, h->w_cap);
      h->Xb = dalloc<double>(h, h->x_cap);
      if (h->multi) {
        // the tangent column of the lockstep runs on its own stream with its own scratch
        HIPCHK(hipStreamCreateWithFlags(&h->s_side, hipStreamNonBlocking));
        HIPCHK(hipStreamCreateWithFlags(&h->s_diag, hipStreamNonBlocking));
        HIPCHK(hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&h->ev_px, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&h->ev_py, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&h->ev_pre, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&h->ev_fin, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&h->ev_post, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&h->ev_diag, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&h->ev_rw, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&h->ev_rest, hipEventDisableTiming));
        h->Wb2 = dalloc<double>(h, h->w_cap);
        h->Xb2 = dalloc<double>(h, h->x_cap);
        h->Urow2 = dalloc<double>(h, h->urow_cap);
        h->skw2 = dalloc<double>(h, h->sk_cap);
        h->tw2 = dalloc<double>(h, 64 * nb + 3 * nb * nb);
      }
      h->lm_cap = std::max<int64_t>(1 << 16, 16 * nt * nt * nterms + 64 * nt);
      h->im_cap = std::max<int64_t>(1 << 20, 64 * nt * nt * nterms + 64 * nt);   // + flat tile lists
      h->im_d = dalloc<int>(h, h->im_cap);
      h->im_h = halloc<int>(h, h->im_cap);
      h->lm_d = dalloc<int64_t>(h, h->lm_cap);
      h->lm_h = halloc<int64_t>(h, h->lm_cap);
      if (h->multi) {
        // the side stream stages the look-ahead updates of whole columns between
        // its recycling points (when full, the host waits for that stream)
        h->im2_cap = 4 * h->im_cap;
        h->lm2_cap = 4 * h->lm_cap;
        h->im2_d = dalloc<int>(h, h->im2_cap);
        h->im2_h = halloc<int>(h, h->im2_cap);
        h->lm2_d = dalloc<int64_t>(h, h->lm2_cap);
        h->lm2_h = halloc<int64_t>(h, h->lm2_cap);
      }
      h->tk_cap = (int)gc;
      h->tk_d = dalloc<QrcpTask>(h, gc);
      h->tk_h = halloc<QrcpTask>(h, gc);
      h->hq_d = dalloc<HqrTask>(h, 6 * gc);
      h->hq_h = halloc<HqrTask>(h, 6 * gc);
      h->tw_stride = (int64_t)((h->smax + 15) / 16) * 256;
      h->Tw = dalloc<double>(h, gc * h->tw_stride);
      h->tr_stride = (int64_t)((kRegQrBig + 15) / 16) * 256;
      h->Tr = dalloc<double>(h, gc * h->tr_stride);
      h->Tau = dalloc<double>(h, gc * (int64_t)kRegQrBig);
      if (h->multi) {   // folded column updates (look-ahead factorisations only)
        h->zst = dalloc<double>(h, h->smax * (int64_t)h->maxrank);
        h->gbuf_cap = gc * (int64_t)h->maxrank * 256;
        // TLR_FOLD_GBUF (doubles) lowers the capacity, so that tests reach the
        // fallback that applies the folded term to the tiles instead
        if (const char* fb = std::getenv("TLR_FOLD_GBUF")) h->gbuf_cap = std::min<int64_t>(h->gbuf_cap, std::atoll(fb));
        h->gbuf = dalloc<double>(h, h->gbuf_cap);
        h->wf_ld = nt * nb;
        h->wf_pcols = h->maxrank;
        h->wf_tcols = 3 * h->maxrank;
        h->wf_cap = h->wf_ld * (h->wf_pcols + h->wf_tcols);
        h->Wf = dalloc<double>(h, h->wf_cap);
        h->zst2_cols = 2 * h->maxrank + kFoldRsumMax;
        h->zst2 = dalloc<double>(h, h->smax * (int64_t)h->zst2_cols);
      }
      h->qr_d = dalloc<int>(h, 2 * gc);
      h->qr_h = halloc_coherent<int>(h, 2 * gc, &h->qr_hd);
      h->aca_d = dalloc<AcaTask>(h, gc);
      h->aca_h = halloc<AcaTask>(h, gc);
      if (o->prec == TLR_PREC_FP32_UPDATES) {
        h->chk_d = dalloc<double>(h, 2 * nt);
        h->chk_h = halloc<double>(h, 2 * nt);
        h->chk_scr = dalloc<double>(h, nb * nb);
      }
      HIPCHK(launch_gaussian(h->omega, nb * h->smax, (uint32_t)o->seed, h->s));
    }
    for (hipEvent_t& e : h->ev) HIPCHK(hipEventCreate(&e));
    reset_info(h);
    HIPCHK(hipStreamSynchronize(h->s));
    h->info.n = n;
    h->info.nb = (int)nb;
    h->info.nt = (int)nt;
    h->info.maxrank = mr;
    h->info.mode = o->mode;
    h->info.device_bytes = h->bytes;
    h->info.bad_tile_i = h->info.bad_tile_j = -1;
    return TLR_OK;
  });
  if (st != TLR_OK) {
    free_all(h);
    delete h;
    return st;
  }
  *out = h;
  return TLR_OK;
}

tlr_status tlr_destroy(tlr_handle_t h) {
  if (!h) return TLR_OK;
  free_all(h);
  delete h;
  return TLR_OK;
}

tlr_status tlr_generate(tlr_handle_t h, const double* d_x, const double* d_y, const double theta[3]) {
  if (!h || !d_x || !d_y || !theta) return TLR_EINVAL;
  return guarded(h, [&]() -> tlr_status {
    MaternParams p{};
    if (!matern_setup(theta[0], theta[1], theta[2], &p, h->h_tab.data())) return TLR_EINVAL;
    HIPCHK(hipMemcpyAsync(h->d_tab, h->h_tab.data(), kTabSize * sizeof(double), hipMemcpyHostToDevice, h->s));
    sync(h);
    p.tab = h->d_tab;
    p.metric = h->o.metric;
    p.radius = h->o.sphere_radius > 0.0 ? h->o.sphere_radius : 6371.0;
    h->mp = p;
    h->x = d_x;
    h->y = d_y;
    for (int i = 0; i < 3; ++i) h->theta[i] = theta[i];
    h->bound = true;
    h->state = 0;
    return TLR_OK;
  });
}

tlr_status tlr_compress(tlr_handle_t h) {
  if (!h) return TLR_EINVAL;
  if (h->dense) return TLR_ENOTIMPL;
  if (!h->bound) return TLR_ESTATE;
  return guarded(h, [&]() -> tlr_status {
    arena_ensure(h);
    for (;;) {
      try {
        if (h->o.flags & TLR_FLAG_ACA) compress_sigma_aca(h); else compress_sigma(h);
        return TLR_OK;
      } catch (const Fail& f) {
        if (!(f.st == TLR_ENOMEM && h->tile_overflow && h->tile_auto)) throw;
        arena_grow(h);
      }
    }
  });
}


tlr_status tlr_potrf(tlr_handle_t h, int64_t* info) {
  if (!h) return TLR_EINVAL;
  if (!h->bound) return TLR_ESTATE;
  if (info) *info = 0;
  return guarded(h, [&]() -> tlr_status {
    prof_reset_pool(h);
    h->state = 0;
    HIPCHK(hipEventRecord(h->ev[0], h->s));
    const tlr_status st = factor_checked(h, false, info);
    if (st != TLR_OK) return st;
    HIPCHK(hipEventRecord(h->ev[1], h->s));
    sync(h);
    h->info.t_factor_ms = elapsed(h->ev[0], h->ev[1]);
    if (!h->dense) rank_stats(h);
    h->state = 2;
    return TLR_OK;
  });
}

tlr_status tlr_loglik(tlr_handle_t h, const double* d_z, double* ll, double* logdet, double* quad) {
  if (!h || !d_z) return TLR_EINVAL;
  if (h->state < 2) return TLR_ESTATE;
  return guarded(h, [&]() -> tlr_status {
    double ld = 0.0, q = 0.0, l = 0.0;
    const double n = (double)h->n;
    for (;;) {
      HIPCHK(hipEventRecord(h->ev[2], h->s));
      solve_forward(h, d_z, &ld, &q);
      HIPCHK(hipEventRecord(h->ev[3], h->s));
      sync(h);
      h->info.t_solve_ms = elapsed(h->ev[2], h->ev[3]);
      l = -0.5 * n * std::log(2.0 * M_PI) - 0.5 * ld - 0.5 * q;
      if (h->state != 2 || !fp32_check_fails(h, l)) break;
      // the FP32 products cannot be shown to hold the tolerance: factor again in FP64
      ++h->info.fp64_retries;
      drop_history(h);
      int64_t info = 0;
      const tlr_status st = factor_checked(h, false, &info);
      if (st != TLR_OK) return st;
      if (!h->dense) rank_stats(h);
    }
    if (ll) *ll = l;
    if (logdet) *logdet = ld;
    if (quad) *quad = q;
    return TLR_OK;
  });
}

tlr_status tlr_sample(tlr_handle_t h, const double* d_eps, double* d_z) {
  if (!h || !d_eps || !d_z || d_eps == d_z) return TLR_EINVAL;
  if (h->state < 2) return TLR_ESTATE;
  return guarded(h, [&]() -> tlr_status {
    const int nt = h->nt, nb = h->nb;
    const int64_t n = h->n;
    for (int j = 0; j < nt; ++j) {
      const int nbj = tile_rows(h, j);
      const int64_t r0 = (int64_t)j * nb;
      const double* Ljj = h->dense ? panel(h, h->Lp, j) : diag_tile(h, j);
      const int64_t ldl = h->dense ? n - r0 : nb;
      HIPCHK(launch_gemv_n(Ljj, ldl, nbj, nbj, d_eps + r0, 1.0, 0.0, d_z + r0, h->s));
    }
    for (int j = 0; j < nt - 1; ++j) {
      const int nbj = tile_rows(h, j);
      const int64_t r0 = (int64_t)j * nb;
      if (h->dense) {
        HIPCHK(launch_gemv_n(panel(h, h->Lp, j) + nbj, n - r0, n - r0 - nbj, nbj, d_eps + r0, 1.0, 1.0,
                             d_z + r0 + nbj, h->s));
      } else {
        LowRankApply a{};
        a.arena = h->arena; a.uoff = h->fam[0].uoff_d; a.voff = h->fam[0].voff_d; a.ranks = h->fam[0].rk_d;
        a.n = n; a.nb = nb; a.nt = nt; a.fixed = j; a.forward = 1; a.v = d_eps; a.out = d_z; a.scale = 1.0;
        a.tws = h->lrtws;
        HIPCHK(launch_lowrank_apply(a, nt - j - 1, h->s, lr_kmax(h, j, true)));
      }
    }
    sync(h);
    return TLR_OK;
  });
}

tlr_status tlr_profile(tlr_handle_t h, int32_t enable) {
  if (!h) return TLR_EINVAL;
  return guarded(h, [&]() -> tlr_status {
    sync(h);
    prof_reset_pool(h);
    if (enable < 0 || enable > 2) return TLR_EINVAL;
    h->prof = enable;
    for (auto& k : h->kst) k = tlr_kstat{};
    return TLR_OK;
  });
}

tlr_status tlr_get_kstats(tlr_handle_t h, tlr_kstat* out) {
  if (!h || !out) return TLR_EINVAL;
  for (int i = 0; i < TLR_K_COUNT; ++i) out[i] = h->kst[i];
  return TLR_OK;
}

tlr_status tlr_get_ranks(tlr_handle_t h, int32_t* host_ranks) {
  if (!h || !host_ranks) return TLR_EINVAL;
  for (size_t i = 0; i < (size_t)h->nt * h->nt; ++i) host_ranks[i] = h->dense ? 0 : h->fam[0].rk[i];
  return TLR_OK;
}

tlr_status tlr_get_tangent_ranks(tlr_handle_t h, int32_t* host_ranks) {
  if (!h || !host_ranks) return TLR_EINVAL;
  if (!h->grad) return TLR_ESTATE;
  for (size_t i = 0; i < (size_t)h->nt * h->nt; ++i) host_ranks[i] = h->dense ? 0 : h->fam[1].rk[i];
  return TLR_OK;
}

tlr_status tlr_get_info(tlr_handle_t h, tlr_info* out) {
  if (!h || !out) return TLR_EINVAL;
  *out = h->info;
  return TLR_OK;
}

tlr_status tlr_get_tile(tlr_handle_t h, int32_t i, int32_t j, double* d_out, int64_t ld) {
  if (!h || !d_out || i < 0 || j < 0 || i >= h->nt || j > i) return TLR_EINVAL;
  if (ld < tile_rows(h, i)) return TLR_EINVAL;
  if (h->state < 1 || (h->dense && h->state < 2)) return TLR_ESTATE;
  return guarded(h, [&]() -> tlr_status {
    const int mi = tile_rows(h, i), mj = tile_rows(h, j);
    if (h->dense) {
      const int64_t ldp = h->n - (int64_t)j * h->nb;
      HIPCHK(launch_copy_block(panel(h, h->Lp, j) + (int64_t)(i - j) * h->nb, ldp, d_out, ld, mi, mj, h->s));
    } else if (i == j) {
      HIPCHK(launch_copy_block(diag_tile(h, i), h->nb, d_out, ld, mi, mj, h->s));
    } else {
      const size_t id = tid_of(h, i, j);
      const int k = h->fam[0].rk[id];
      GemmSeg sg{};
      sg.A = op_contig(h->arena + h->fam[0].uoff[id], h->nb, 0, 0);
      sg.B = op_contig(h->arena + h->fam[0].voff[id], h->nb, 0, 0);
      sg.K = k;
      gemm(h, mi, mj, 1, &sg, d_out, ld, epi_linear(1.0, 0.0));
    }
    sync(h);
    return TLR_OK;
  });
}

tlr_status tlr_covariance_block(tlr_handle_t h, int64_t r0, int64_t m, int64_t c0, int64_t k, int32_t deriv,
                                double* d_out, int64_t ld) {
  if (!h || !d_out || m < 0 || k < 0 || r0 < 0 || c0 < 0 || r0 + m > h->n || c0 + k > h->n || ld < m)
    return TLR_EINVAL;
  if (!h->bound) return TLR_ESTATE;
  if (deriv < 0 || deriv > 2) return TLR_EINVAL;
  return guarded(h, [&]() -> tlr_status {
    MaternParams p = h->mp;
    p.dparam = deriv == 2 ? kDerivNu : kDerivBeta;
    HIPCHK(launch_matern_block(p, h->x, h->y, r0, m, c0, k, d_out, ld, deriv != 0, h->s));
    sync(h);
    return TLR_OK;
  });
}

}  // extern "C"

namespace {
// l and the score of one theta parameter besides sigma^2: grad = (dl/dsigma^2,
// dl/dtheta_d), theta_d = beta (dparam kDerivBeta) or nu (kDerivNu); the
// tangent factorisation and the quadratic term both take their dSigma from
// the Matérn generation with that derivative selected.
tlr_status loglik_grad_impl(tlr_handle_t h, const double* d_x, const double* d_y, const double* d_z,
                            const double theta[3], double* ll, double grad[2], int64_t* info, int dparam) {
  if (!h || !d_x || !d_y || !d_z || !theta || !grad) return TLR_EINVAL;
  if (!h->grad) return TLR_ESTATE;
  if (info) *info = 0;
  tlr_status st = tlr_generate(h, d_x, d_y, theta);
  if (st != TLR_OK) return st;
  h->mp.dparam = dparam;
  return guarded(h, [&]() -> tlr_status {
    double ld = 0.0, q = 0.0;
    const double n = (double)h->n;
    for (;;) {
      prof_reset_pool(h);
      h->state = 0;
      HIPCHK(hipEventRecord(h->ev[0], h->s));
      const tlr_status fst = factor_checked(h, true, info);
      if (fst != TLR_OK) return fst;
      HIPCHK(hipEventRecord(h->ev[1], h->s));
      sync(h);
      h->info.t_factor_ms = elapsed(h->ev[0], h->ev[1]);
      if (!h->dense) rank_stats(h);
      h->state = 3;
      HIPCHK(hipEventRecord(h->ev[2], h->s));
      const size_t e_s = prof_mark(h);
      solve_forward(h, d_z, &ld, &q);
      if (!fp32_check_fails(h, -0.5 * n * std::log(2.0 * M_PI) - 0.5 * ld - 0.5 * q)) {
        solve_backward(h);
        prof_add(h, TLR_K_SOLVE, e_s, 0.0, 0.0);
        break;
      }
      // the FP32 products cannot be shown to hold the tolerance: factor again in FP64
      ++h->info.fp64_retries;
      drop_history(h);
    }
    HIPCHK(hipEventRecord(h->ev[3], h->s));
    const size_t e_q = prof_mark(h);
    // a^T dSigma/dbeta a over all pairs; partial sums in the split-K workspace
    const int64_t nblk = pair_quad_blocks(h->n);
    if (nblk > h->sk_cap) NOMEM("pair-sum partials");
    HIPCHK(launch_pair_quad(h->mp, h->x, h->y, h->vec + 2 * h->n, h->n, h->skw, h->scal + 2 * h->nt + 1, h->s));
    prof_add(h, TLR_K_GRADQ, e_q, (double)h->n * (double)(h->n - 1) / 2.0, 24.0 * h->n);
    HIPCHK(hipEventRecord(h->ev[1], h->s));
    HIPCHK(hipMemcpyAsync(h->h_scal, h->scal, (2 * h->nt + 2) * sizeof(double), hipMemcpyDeviceToHost, h->s));
    sync(h);
    h->info.t_solve_ms = elapsed(h->ev[2], h->ev[3]);
    h->info.t_grad_ms = elapsed(h->ev[3], h->ev[1]);
    double trace = 0.0;
    for (int j = 0; j < h->nt; ++j) trace += h->h_scal[h->nt + j];
    const double qf = h->h_scal[2 * h->nt + 1];
    if (ll) *ll = -0.5 * n * std::log(2.0 * M_PI) - 0.5 * ld - 0.5 * q;
    grad[0] = (q - n) / (2.0 * h->theta[0]);
    grad[1] = -0.5 * trace + 0.5 * qf;
    return TLR_OK;
  });
}
}  // namespace

extern "C" tlr_status tlr_loglik_grad(tlr_handle_t h, const double* d_x, const double* d_y, const double* d_z,
                                      const double theta[3], double* ll, double grad[2], int64_t* info) {
  return loglik_grad_impl(h, d_x, d_y, d_z, theta, ll, grad, info, kDerivBeta);
}

extern "C" tlr_status tlr_loglik_grad3(tlr_handle_t h, const double* d_x, const double* d_y, const double* d_z,
                                       const double theta[3], double* ll, double grad[3], int64_t* info) {
  if (!grad) return TLR_EINVAL;
  double g[2];
  tlr_status st = loglik_grad_impl(h, d_x, d_y, d_z, theta, ll, g, info, kDerivBeta);
  if (st != TLR_OK) return st;
  grad[0] = g[0];
  grad[1] = g[1];
  // the same evaluation with the tangent in nu; l, log|Sigma| and q are kept
  // from the first pass
  st = loglik_grad_impl(h, d_x, d_y, d_z, theta, nullptr, g, info, kDerivNu);
  h->mp.dparam = kDerivBeta;
  if (st != TLR_OK) return st;
  grad[2] = g[1];
  return TLR_OK;
}

extern "C" tlr_status tlr_loglik_grad_batched(int32_t nfields, const tlr_handle_t* hs, const double* const* d_x,
                                              const double* const* d_y, const double* const* d_z,
                                              const double* theta, double* ll, double* grad, int64_t* info,
                                              int32_t* status, int32_t nthreads) {
  if (nfields < 0) return TLR_EINVAL;
  if (nfields == 0) return TLR_OK;
  if (!hs || !d_x || !d_y || !d_z || !theta || !grad) return TLR_EINVAL;
  {
    std::vector<tlr_handle_t> seen(hs, hs + nfields);
    for (tlr_handle_t x : seen)
      if (!x) return TLR_EINVAL;
    std::sort(seen.begin(), seen.end());
    if (std::adjacent_find(seen.begin(), seen.end()) != seen.end()) return TLR_EINVAL;   // one handle, one field
  }
  const int T = std::max(1, std::min<int>(nthreads <= 0 ? 4 : nthreads, std::min<int>(nfields, 64)));
  std::atomic<int> next{0};
  std::vector<tlr_status> st((size_t)nfields, TLR_OK);
  std::vector<std::string> msg((size_t)nfields);   // the error text is per thread: keep each field's
  auto worker = [&]() {
    int dev = -1;
    for (;;) {
      const int f = next.fetch_add(1);
      if (f >= nfields) break;
      if (hs[f]->device != dev) {
        dev = hs[f]->device;
        if (hipSetDevice(dev) != hipSuccess) {
          (void)hipGetLastError();
          dev = -1;   // not switched: the next field tries again
          st[f] = TLR_EHIP;
          continue;
        }
      }
      int64_t inf = 0;
      st[f] = tlr_loglik_grad(hs[f], d_x[f], d_y[f], d_z[f], theta + 3 * (size_t)f, ll ? ll + f : nullptr,
                              grad + 2 * (size_t)f, &inf);
      if (info) info[f] = inf;
      if (st[f] != TLR_OK) msg[f] = g_last_error;
    }
  };
  std::vector<std::thread> pool;
  try {
    for (int t = 1; t < T; ++t) pool.emplace_back(worker);
  } catch (const std::system_error&) {
    // fewer threads than asked: the rest of the work falls to those started
  }
  worker();
  for (std::thread& t : pool) t.join();
  tlr_status first = TLR_OK;
  for (int f = 0; f < nfields; ++f) {
    if (status) status[f] = st[f];
    if (first == TLR_OK && st[f] != TLR_OK) {
      first = st[f];
      snprintf(g_last_error, sizeof(g_last_error), "%s", msg[f].c_str());
    }
  }
  return first;
}
