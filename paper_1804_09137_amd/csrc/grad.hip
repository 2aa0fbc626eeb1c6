// Gradient pieces of the score dl/dbeta = -1/2 tr(Sigma^{-1} dSigma) +
// 1/2 a^T dSigma a, a = Sigma^{-1} z (the textbook score of the Gaussian
// likelihood Eq. (1); the paper's optimiser is derivative-free).
//
//  * pair_quad_kernel: a^T dSigma/dbeta a = sum_{a,b} a_a a_b dC/dbeta(r_ab),
//    entries regenerated on the fly (never stored), lower-triangle blocks of
//    128 x 128 pairs, one partial per workgroup, reduced in a fixed order.
//  * diag_trace_kernel + phi_kernel: tangent of the diagonal Cholesky step,
//    M = L^{-1} dC L^{-T},  Phi(M) = tril(M) with the diagonal halved,
//    and tr(M) (the tile's share of d log|Sigma|).
#include "kernels.h"
#include "matern.h"
#include "grad.h"

namespace tlrk {

constexpr int kPB = 128;

__global__ void __launch_bounds__(256) pair_quad_kernel(MaternParams p, const double* __restrict__ x,
                                                        const double* __restrict__ y, const double* __restrict__ a,
                                                        int64_t n, int64_t nblk, double* __restrict__ partial) {
  __shared__ double rx[kPB], ry[kPB], ra[kPB], cx[kPB], cy[kPB], ca[kPB];
  __shared__ double red[4];
  const int64_t b = blockIdx.x;
  // lower-triangle block index b -> (I, J), I >= J
  int64_t I = (int64_t)((sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
  while ((I + 1) * (I + 2) / 2 <= b) ++I;
  while (I * (I + 1) / 2 > b) --I;
  const int64_t J = b - I * (I + 1) / 2;
  const int tid = threadIdx.x;
  const int64_t r0 = I * kPB, c0 = J * kPB;
  if (tid < kPB) {
    const int64_t r = r0 + tid;
    rx[tid] = r < n ? x[r] : 0.0;
    ry[tid] = r < n ? y[r] : 0.0;
    ra[tid] = r < n ? a[r] : 0.0;
  } else {
    const int t = tid - kPB;
    const int64_t c = c0 + t;
    cx[t] = c < n ? x[c] : 0.0;
    cy[t] = c < n ? y[c] : 0.0;
    ca[t] = c < n ? a[c] : 0.0;
  }
  __syncthreads();
  double s = 0.0;
  const bool diag = (I == J);
  for (int e = tid; e < kPB * kPB; e += 256) {
    const int i = e % kPB, j = e / kPB;
    if (diag && i <= j) continue;
    if (r0 + i >= n || c0 + j >= n) continue;
    double cv, dv;
    matern_eval<true>(p, point_dist(p, rx[i], ry[i], cx[j], cy[j]), cv, dv);
    s += ra[i] * ca[j] * dv;
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((tid & 63) == 0) red[tid >> 6] = s;
  __syncthreads();
  if (tid == 0) partial[b] = 2.0 * ((red[0] + red[1]) + (red[2] + red[3]));
  (void)nblk;
}

// Sums partial[0 .. cnt) into out[0] with one workgroup, fixed order per thread.
__global__ void __launch_bounds__(256) sum_kernel(const double* __restrict__ partial, int64_t cnt, double* out) {
  __shared__ double red[4];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < cnt; i += 256) s += partial[i];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) *out = (red[0] + red[1]) + (red[2] + red[3]);
}

int64_t pair_quad_blocks(int64_t n) {
  const int64_t nbk = (n + kPB - 1) / kPB;
  return nbk * (nbk + 1) / 2;
}

hipError_t launch_pair_quad(const MaternParams& p, const double* x, const double* y, const double* a, int64_t n,
                            double* partial, double* out, hipStream_t s) {
  const int64_t nblk = pair_quad_blocks(n);
  if (nblk > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(pair_quad_kernel, dim3((unsigned)nblk), dim3(256), 0, s, p, x, y, a, n, nblk, partial);
  hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(256), 0, s, partial, nblk, out);
  return hipGetLastError();
}

// M (m x m, ld) <- Phi(M) = tril(M) with halved diagonal; *trace_out = tr(M).
// trace of the m x m block (one workgroup, fixed summation order), read
// before phi_kernel halves the diagonal
__global__ void __launch_bounds__(256) diag_trace_kernel(const double* __restrict__ M, int64_t ld, int64_t m,
                                                         double* trace_out) {
  __shared__ double red[4];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < m; i += 256) s += M[i * ld + i];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) *trace_out = (red[0] + red[1]) + (red[2] + red[3]);
}

// Phi(M): zero above the diagonal, halve the diagonal; block (x, k) takes
// rows 256 x.. of column k
__global__ void __launch_bounds__(256) phi_kernel(double* __restrict__ M, int64_t ld, int64_t m) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t k = blockIdx.y;
  if (i > k || k >= m) return;
  double* p = M + k * ld + i;
  *p = (i == k) ? 0.5 * *p : 0.0;
}

hipError_t launch_phi_trace(double* M, int64_t ld, int64_t m, double* trace_out, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(diag_trace_kernel, dim3(1), dim3(256), 0, s, M, ld, m, trace_out);
  hipLaunchKernelGGL(phi_kernel, dim3((unsigned)((m + 255) / 256), (unsigned)m), dim3(256), 0, s, M, ld, m);
  return hipGetLastError();
}

}  // namespace tlrk
