// Kriging prediction at new locations (Section III, Eq. (pred3)) from a
// factor of Sigma_22 held by a handle:
//   Z_1 = Sigma_12 Sigma_22^{-1} Z_2,
// computed as a = L^{-T} L^{-1} Z_2 (the forward and backward solves over the
// dense or TLR factor) followed by Z_1[i] = sum_b C(d(s_new_i, s_b)) a_b, the
// cross-covariance Sigma_12 generated on the fly and never stored.
// Optionally the conditional variance of Eq. (pred2),
//   Var[Z_1 | Z_2]_ii = C(0) - ||L^{-1} Sigma_21[:, i]||^2,
// by one forward solve per new location.
#include "handle.h"
#include "matern.h"

namespace tlrk {

constexpr int kPredChunk = 4096;   // observed points per workgroup

// partial[i * nchunk + c] = sum over chunk c of C(d(new_i, s_b)) a_b
__global__ void __launch_bounds__(256) predict_partial_kernel(MaternParams p, const double* __restrict__ xn,
                                                              const double* __restrict__ yn,
                                                              const double* __restrict__ x,
                                                              const double* __restrict__ y,
                                                              const double* __restrict__ a, int64_t n,
                                                              int64_t nchunk, double* __restrict__ partial) {
  __shared__ double red[4];
  const int64_t i = blockIdx.y, c = blockIdx.x;
  const double xi = xn[i], yi = yn[i];
  const int64_t b0 = c * kPredChunk;
  const int64_t b1 = (b0 + kPredChunk < n) ? b0 + kPredChunk : n;
  double s = 0.0;
  for (int64_t b = b0 + threadIdx.x; b < b1; b += 256) {
    double cv, dv;
    matern_eval<false>(p, point_dist(p, xi, yi, x[b], y[b]), cv, dv);
    s += cv * a[b];
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) partial[i * nchunk + c] = (red[0] + red[1]) + (red[2] + red[3]);
}

// out[i] = sum_c partial[i * nchunk + c], in chunk order (one thread per i)
__global__ void __launch_bounds__(256) predict_sum_kernel(const double* __restrict__ partial, int64_t m,
                                                          int64_t nchunk, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= m) return;
  double s = 0.0;
  for (int64_t c = 0; c < nchunk; ++c) s += partial[i * nchunk + c];
  out[i] = s;
}

// col[b] = C(d(new_i, s_b)) for b < n (column i of Sigma_21)
__global__ void __launch_bounds__(256) cross_cov_kernel(MaternParams p, double xi, double yi,
                                                        const double* __restrict__ x, const double* __restrict__ y,
                                                        int64_t n, double* __restrict__ col) {
  const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (b >= n) return;
  double cv, dv;
  matern_eval<false>(p, point_dist(p, xi, yi, x[b], y[b]), cv, dv);
  col[b] = cv;
}

}  // namespace tlrk

using namespace tlrk;
using namespace tlri;

extern "C" tlr_status tlr_predict(tlr_handle_t h, const double* d_z, int64_t m, const double* d_xnew,
                                  const double* d_ynew, double* d_pred, double* d_var) {
  if (!h || !d_z || m < 0 || (m > 0 && (!d_xnew || !d_ynew || !d_pred))) return TLR_EINVAL;
  if (h->state < 2) return TLR_ESTATE;
  if (m == 0) return TLR_OK;
  if (m > 65535) return TLR_EINVAL;
  return guarded(h, [&]() -> tlr_status {
    const int64_t n = h->n;
    double ld = 0.0, q = 0.0;
    solve_forward(h, d_z, &ld, &q);
    solve_backward(h);
    const double* alpha = h->vec + 2 * n;
    const int64_t nchunk = (n + kPredChunk - 1) / kPredChunk;
    if (m * nchunk > h->sk_cap) NOMEM("prediction partial sums");
    hipLaunchKernelGGL(predict_partial_kernel, dim3((unsigned)nchunk, (unsigned)m), dim3(256), 0, h->s, h->mp,
                       d_xnew, d_ynew, h->x, h->y, alpha, n, nchunk, h->skw);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(predict_sum_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, h->s, h->skw, m, nchunk,
                       d_pred);
    HIPCHK(hipGetLastError());
    if (d_var) {
      // Eq. (pred2): C(0) - ||L^{-1} c_i||^2, c_i = Sigma_21[:, i]
      std::vector<double> xs((size_t)m), ys((size_t)m), var((size_t)m);
      HIPCHK(hipMemcpyAsync(xs.data(), d_xnew, m * sizeof(double), hipMemcpyDeviceToHost, h->s));
      HIPCHK(hipMemcpyAsync(ys.data(), d_ynew, m * sizeof(double), hipMemcpyDeviceToHost, h->s));
      sync(h);
      double* col = h->vec + 3 * n;
      for (int64_t i = 0; i < m; ++i) {
        hipLaunchKernelGGL(cross_cov_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, h->s, h->mp, xs[i],
                           ys[i], h->x, h->y, n, col);
        HIPCHK(hipGetLastError());
        solve_forward(h, col, &ld, &q);
        var[(size_t)i] = h->mp.sigma2 - q;
      }
      HIPCHK(hipMemcpyAsync(d_var, var.data(), m * sizeof(double), hipMemcpyHostToDevice, h->s));
    }
    sync(h);
    return TLR_OK;
  });
}
