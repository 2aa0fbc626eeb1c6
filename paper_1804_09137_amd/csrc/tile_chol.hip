// Blocked Cholesky and inverse of one dense diagonal tile (the POTRF step of
// the tile Cholesky, Section V), built from the MFMA GEMM and the 64 x 64
// in-LDS factorisation.
#include "chol.h"
#include "kernels.h"

namespace tlrk {

namespace {
Operand contig(const double* base, int64_t ld, int64_t r0, int64_t c0) {
  Operand o{};
  o.base = base;
  o.ld = ld;
  o.r0 = r0;
  o.c0 = c0;
  o.layout = kContig;
  return o;
}
Operand contigT(const double* base, int64_t ld, int64_t r0, int64_t c0) {
  Operand o = contig(base, ld, r0, c0);
  o.layout = kContigT;
  return o;
}
GemmEpi linear(double alpha, double beta) {
  GemmEpi e{};
  e.kind = kEpiLinear;
  e.alpha = alpha;
  e.beta = beta;
  return e;
}
}  // namespace

#define TLRK_TRY(x)                          \
  do {                                       \
    hipError_t e_ = (x);                     \
    if (e_ != hipSuccess) return e_;         \
  } while (0)

hipError_t tile_potrf_inv(double* T, int64_t ld, int64_t m, double* Inv, int64_t ldi, unsigned long long* info,
                          int64_t row0, double* work, hipStream_t s) {
  constexpr int64_t W = 64;
  for (int64_t c0 = 0; c0 < m; c0 += W) {
    const int64_t wt = (m - c0 < W) ? m - c0 : W;
    if (c0 > 0) {  // left-looking update of the block column
      GemmSeg sg{};
      sg.A = contig(T, ld, c0, 0);
      sg.B = contig(T, ld, c0, 0);
      sg.K = c0;
      TLRK_TRY(launch_gemm(m - c0, wt, 1, &sg, T + c0 * ld + c0, ld, linear(-1.0, 1.0), nullptr, 1, nullptr, s));
    }
    TLRK_TRY(launch_potrf_small(T + c0 * ld + c0, ld, (int)wt, Inv + c0 * ldi + c0, ldi, info, row0 + c0, s));
    if (c0 + wt < m) {  // panel below: X = P L_tt^{-T}, in place (one workgroup column covers N = wt)
      GemmSeg sg{};
      sg.A = contig(T, ld, c0 + wt, c0);
      sg.B = contig(Inv + c0 * ldi + c0, ldi, 0, 0);
      sg.K = wt;
      TLRK_TRY(launch_gemm(m - c0 - wt, wt, 1, &sg, T + c0 * ld + c0 + wt, ld, linear(1.0, 0.0), nullptr, 1,
                           nullptr, s));
    }
  }
  // the block products below read whole squares of Inv: clear its upper part
  TLRK_TRY(launch_zero_upper(Inv, ldi, m, s));
  // inverse by block rows: Inv[t, <t] = -Inv_tt (T[t, <t] Inv[<t, <t])
  for (int64_t c0 = W; c0 < m; c0 += W) {
    const int64_t wt = (m - c0 < W) ? m - c0 : W;
    GemmSeg a{};
    a.A = contig(T, ld, c0, 0);
    a.B = contigT(Inv, ldi, 0, 0);
    a.K = c0;
    TLRK_TRY(launch_gemm(wt, c0, 1, &a, work, wt, linear(1.0, 0.0), nullptr, 1, nullptr, s));
    GemmSeg b{};
    b.A = contig(Inv + c0 * ldi + c0, ldi, 0, 0);
    b.B = contigT(work, wt, 0, 0);
    b.K = wt;
    TLRK_TRY(launch_gemm(wt, c0, 1, &b, Inv + c0, ldi, linear(-1.0, 0.0), nullptr, 1, nullptr, s));
  }
  TLRK_TRY(launch_zero_upper(T, ld, m, s));
  return hipSuccess;
}

}  // namespace tlrk
