// Dense tile kernels of the Cholesky-based likelihood (Section III; task list
// of Section VI): small-block Cholesky with inverse, triangle clean-up,
// log-determinant reduction, matrix-vector products for the triangular solves.
#include "kernels.h"
#include "chol.h"

namespace tlrk {

// Factor the w x w (w <= 64) diagonal block at A (column-major, lda) in place
// (lower Cholesky), and write its inverse (lower, zero above) to Inv (ldi).
// A pivot that is not > 0 (or NaN) records row0 + c + 1 in *info (atomicMin
// over 1-based rows; *info must start at INT64_MAX) and the factorisation
// continues with the pivot replaced by 1 so that no NaN/inf is produced.
__global__ void __launch_bounds__(256) potrf_small_kernel(double* __restrict__ A, int64_t lda, int w,
                                                          double* __restrict__ Inv, int64_t ldi,
                                                          unsigned long long* info, int64_t row0) {
  __shared__ double L[64][65];
  __shared__ double X[64][65];
  const int tid = threadIdx.x;
  const int li = tid & 63;    // row handled by this lane
  const int kq = tid >> 6;    // this wave's columns: k = kq + 4 s
  for (int k = kq; k < w; k += 4) {
    L[li][k] = (li < w && li >= k) ? A[(int64_t)k * lda + li] : 0.0;
    X[li][k] = 0.0;
  }
  __syncthreads();
  // right-looking: scale column c, then rank-1 update of the lower part
  for (int c = 0; c < w; ++c) {
    double d = L[c][c];
    const bool bad = !(d > 0.0);
    if (bad) d = 1.0;
    const double sc = sqrt(d);
    const double is = 1.0 / sc;
    __syncthreads();   // every thread has read L[c][c]
    if (tid == 0) {
      if (bad) atomicMin(info, (unsigned long long)(row0 + c + 1));
      L[c][c] = sc;
    }
    if (tid < 64 && li > c && li < w) L[li][c] *= is;
    __syncthreads();
    const double lic = (li > c && li < w) ? L[li][c] : 0.0;
    for (int k = c + 1 + ((kq - c - 1) & 3); k < w; k += 4)
      if (li >= k) L[li][k] -= lic * L[k][c];
    __syncthreads();
  }
  // X = L^{-1} by rows: X[i][k] = (delta_ik - sum_{k <= t < i} L[i][t] X[t][k]) / L[i][i];
  // the four waves split the sum over t, lane k owns column k
  __shared__ double part[4][64];
  for (int i = 0; i < w; ++i) {
    const int k = li;
    double acc = 0.0;
    if (k < i)
      for (int t = k + kq; t < i; t += 4) acc += L[i][t] * X[t][k];
    part[kq][k] = acc;
    __syncthreads();
    if (tid < 64 && k <= i) {
      const double s = part[0][k] + part[1][k] + part[2][k] + part[3][k];
      X[i][k] = ((k == i ? 1.0 : 0.0) - s) / L[i][i];
    }
    __syncthreads();
  }
  for (int k = kq; k < w; k += 4) {
    if (li < w) {
      if (li >= k) A[(int64_t)k * lda + li] = L[li][k];
      Inv[(int64_t)k * ldi + li] = (li >= k) ? X[li][k] : 0.0;
    }
  }
}

hipError_t launch_potrf_small(double* A, int64_t lda, int w, double* Inv, int64_t ldi,
                              unsigned long long* info, int64_t row0, hipStream_t s) {
  if (w < 1 || w > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(potrf_small_kernel, dim3(1), dim3(256), 0, s, A, lda, w, Inv, ldi, info, row0);
  return hipGetLastError();
}

// Zero the strictly upper part of an m x m column-major block.
__global__ void zero_upper_kernel(double* A, int64_t lda, int64_t m) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t k = blockIdx.y;
  if (i < k && k < m) A[k * lda + i] = 0.0;
}

hipError_t launch_zero_upper(double* A, int64_t lda, int64_t m, hipStream_t s) {
  if (m <= 1) return hipSuccess;
  hipLaunchKernelGGL(zero_upper_kernel, dim3((unsigned)((m + 255) / 256), (unsigned)m), dim3(256), 0, s, A, lda, m);
  return hipGetLastError();
}

// out[b * ldo + a] = in[b * ldi + a], a < m, b < ncol
__global__ void copy_block_kernel(const double* __restrict__ in, int64_t ldi, double* __restrict__ out, int64_t ldo,
                                  int64_t m) {
  const int64_t a = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t b = blockIdx.y;
  if (a < m) out[b * ldo + a] = in[b * ldi + a];
}

hipError_t launch_copy_block(const double* in, int64_t ldi, double* out, int64_t ldo, int64_t m, int64_t ncol,
                             hipStream_t s) {
  if (m <= 0 || ncol <= 0) return hipSuccess;
  for (int64_t c = 0; c < ncol; c += 65535) {
    const int64_t nc = ncol - c < 65535 ? ncol - c : 65535;
    hipLaunchKernelGGL(copy_block_kernel, dim3((unsigned)((m + 255) / 256), (unsigned)nc), dim3(256), 0, s,
                       in + c * ldi, ldi, out + c * ldo, ldo, m);
  }
  return hipGetLastError();
}

// Sum of log of the diagonal of an m x m block: one workgroup, wave
// reductions; result written to *out (no accumulation, deterministic).
__global__ void __launch_bounds__(256) logdiag_kernel(const double* __restrict__ A, int64_t lda, int64_t m,
                                                      double* out) {
  __shared__ double part[4];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < m; i += 256) s += log(A[i * lda + i]);
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) *out = (part[0] + part[1]) + (part[2] + part[3]);
}

hipError_t launch_logdiag(const double* A, int64_t lda, int64_t m, double* out, hipStream_t s) {
  hipLaunchKernelGGL(logdiag_kernel, dim3(1), dim3(256), 0, s, A, lda, m, out);
  return hipGetLastError();
}

// y[0:m] = beta * y + alpha * A[0:m, 0:k] x   (A column-major, one thread per row)
__global__ void __launch_bounds__(256) gemv_n_kernel(const double* __restrict__ A, int64_t lda, int64_t m, int64_t k,
                                                     const double* __restrict__ x, double alpha, double beta,
                                                     double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= m) return;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int64_t c = 0;
  for (; c + 4 <= k; c += 4) {
    a0 += A[c * lda + i] * x[c];
    a1 += A[(c + 1) * lda + i] * x[c + 1];
    a2 += A[(c + 2) * lda + i] * x[c + 2];
    a3 += A[(c + 3) * lda + i] * x[c + 3];
  }
  for (; c < k; ++c) a0 += A[c * lda + i] * x[c];
  const double v = (a0 + a1) + (a2 + a3);
  y[i] = (beta == 0.0 ? 0.0 : beta * y[i]) + alpha * v;
}

hipError_t launch_gemv_n(const double* A, int64_t lda, int64_t m, int64_t k, const double* x, double alpha,
                         double beta, double* y, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(gemv_n_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, A, lda, m, k, x, alpha,
                     beta, y);
  return hipGetLastError();
}

// y[0:k] = beta * y + alpha * A[0:m, 0:k]^T x : one workgroup per column.
__global__ void __launch_bounds__(256) gemv_t_kernel(const double* __restrict__ A, int64_t lda, int64_t m,
                                                     const double* __restrict__ x, double alpha, double beta,
                                                     double* __restrict__ y) {
  __shared__ double part[4];
  const int64_t c = blockIdx.x;
  const double* a = A + c * lda;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < m; i += 256) s += a[i] * x[i];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double v = (part[0] + part[1]) + (part[2] + part[3]);
    y[c] = (beta == 0.0 ? 0.0 : beta * y[c]) + alpha * v;
  }
}

hipError_t launch_gemv_t(const double* A, int64_t lda, int64_t m, int64_t k, const double* x, double alpha,
                         double beta, double* y, hipStream_t s) {
  if (k <= 0) return hipSuccess;
  hipLaunchKernelGGL(gemv_t_kernel, dim3((unsigned)k), dim3(256), 0, s, A, lda, m, x, alpha, beta, y);
  return hipGetLastError();
}

// Dot product of two length-m vectors (one workgroup) -> *out.
__global__ void __launch_bounds__(256) dot_kernel(const double* __restrict__ a, const double* __restrict__ b,
                                                  int64_t m, double* out) {
  __shared__ double part[4];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < m; i += 256) s += a[i] * b[i];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) *out = (part[0] + part[1]) + (part[2] + part[3]);
}

hipError_t launch_dot(const double* a, const double* b, int64_t m, double* out, hipStream_t s) {
  hipLaunchKernelGGL(dot_kernel, dim3(1), dim3(256), 0, s, a, b, m, out);
  return hipGetLastError();
}

}  // namespace tlrk

namespace tlrk {

// A[0:m, 0:ncol] = value (column-major, lda); a plain kernel rather than a
// memset so the operation can sit inside a captured graph.
__global__ void fill_kernel(double* A, int64_t lda, int64_t m, double value) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < m) A[(int64_t)blockIdx.y * lda + i] = value;
}

hipError_t launch_fill(double* A, int64_t lda, int64_t m, int64_t ncol, double value, hipStream_t s) {
  if (m <= 0 || ncol <= 0) return hipSuccess;
  for (int64_t c = 0; c < ncol; c += 65535) {
    const int64_t nc = ncol - c < 65535 ? ncol - c : 65535;
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((m + 255) / 256), (unsigned)nc), dim3(256), 0, s, A + c * lda,
                       lda, m, value);
  }
  return hipGetLastError();
}

}  // namespace tlrk

namespace tlrk {

__global__ void identity_kernel(double* A, int64_t lda, int64_t m) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < m) A[i * lda + i] = 1.0;
}

// diagonal of the m x m block A set to 1 (the rest is left as is)
hipError_t launch_identity(double* A, int64_t lda, int64_t m, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(identity_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, A, lda, m);
  return hipGetLastError();
}

}  // namespace tlrk
