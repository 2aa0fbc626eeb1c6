// Dense tile kernels of the Cholesky-based likelihood (Section III; task list
// of Section VI): small-block Cholesky with inverse, triangle clean-up,
// log-determinant reduction, matrix-vector products for the triangular solves.
#include "kernels.h"
#include "chol.h"
#include "wave.h"

namespace tlrk {

// Cholesky factor L and inverse L^{-1} of a w x w block (w <= 64) by one
// wave.  Both halves are 64 steps of register rank-1 updates whose other
// operand is broadcast from LDS:
//   factor: lane i keeps row i of the matrix; at step c the scaled column c
//     is published and every lane updates its entries right of c (entries
//     right of the diagonal are never read as results);
//   inverse: lane k keeps column k of X = L^{-1}, solved forward: at step t
//     its X[t][k] is final, and every entry below it takes -L[r][t] X[t][k].
// Rows and columns beyond w are padded with the identity.  A pivot that is
// not > 0 (or NaN) is replaced by 1 and reported as info = row0 + c + 1
// (atomicMin over calls; *info starts at the maximum).
namespace {
// v[k] -= s * b[k] for k in (c, 64), b in LDS
template <int C>
__device__ __forceinline__ void rank1_lds(double (&v)[64], double sv, const double* b) {
#pragma unroll
  for (int k = C + 1; k < 64; ++k) v[k] -= sv * b[k];
}
template <int C>
struct Potrf64 {
  __device__ __forceinline__ static void factor(double (&a)[64], double* col, int i, int w, int& bad) {
    double d = wave::read(a[C], C);
    if (!(d > 0.0)) {
      if (C < w && bad == 0) bad = C + 1;
      d = 1.0;
    }
    // 1 / sqrt(d) from the hardware estimate and two Newton-Raphson steps
    // (error ~1 ulp): a division here is expanded inside a per-lane branch,
    // and 64 such branches around the live row defeat register allocation
    double is = __builtin_amdgcn_rsq(d);
    is = is * (1.5 - 0.5 * d * is * is);
    is = is * (1.5 - 0.5 * d * is * is);
    const double sc = d * is;
    a[C] = (i > C) ? a[C] * is : (i == C ? sc : a[C]);
    col[i] = a[C];
    __syncthreads();
    rank1_lds<C>(a, a[C], col);
    __syncthreads();
    Potrf64<C + 1>::factor(a, col, i, w, bad);
  }
  // Ls: rows of L (ld 65), row t at Ls + t * 65
  __device__ __forceinline__ static void inverse(double (&x)[64], const double* Ls, int i) {
    x[C] = ((C == i ? 1.0 : 0.0) - x[C]) * (1.0 / Ls[C * 65 + C]);
    // entries r > C of column i: x[r] += L[r][C] x[C] (negated at finalisation)
#pragma unroll
    for (int r = C + 1; r < 64; ++r) x[r] += Ls[r * 65 + C] * x[C];
    Potrf64<C + 1>::inverse(x, Ls, i);
  }
};
template <>
struct Potrf64<64> {
  __device__ __forceinline__ static void factor(double (&)[64], double*, int, int, int&) {}
  __device__ __forceinline__ static void inverse(double (&)[64], const double*, int) {}
};
}  // namespace

__global__ void __launch_bounds__(64) potrf_small_kernel(double* __restrict__ A, int64_t lda, int w,
                                                         double* __restrict__ Inv, int64_t ldi,
                                                         unsigned long long* info, int64_t row0) {
  __shared__ double col[64];
  __shared__ double Ls[64 * 65];
  const int i = threadIdx.x;
  // the block goes through LDS (coalesced column reads); each lane then
  // takes its row, padded with the identity
  for (int k = 0; k < 64; ++k)
    Ls[i * 65 + k] = (i < w && k < w) ? (k <= i ? A[(int64_t)k * lda + i] : 0.0) : (i == k ? 1.0 : 0.0);
  __syncthreads();
  double a[64];
#pragma unroll
  for (int k = 0; k < 64; ++k) a[k] = Ls[i * 65 + k];
  int bad = 0;
  Potrf64<0>::factor(a, col, i, w, bad);
  if (bad && i == 0) atomicMin(info, (unsigned long long)(row0 + bad));
#pragma unroll
  for (int k = 0; k < 64; ++k) Ls[i * 65 + k] = (k <= i) ? a[k] : 0.0;
  __syncthreads();
  for (int k = 0; k < w; ++k)
    if (i < w && k <= i) A[(int64_t)k * lda + i] = Ls[i * 65 + k];
  // x[r] accumulates sum_{t<r} L[r][t] X[t][i] until step r finalises it
  double x[64];
#pragma unroll
  for (int r = 0; r < 64; ++r) x[r] = 0.0;
  Potrf64<0>::inverse(x, Ls, i);
  __syncthreads();
  // transpose through LDS so that the stores below are coalesced
#pragma unroll
  for (int r = 0; r < 64; ++r) Ls[r * 65 + i] = x[r];
  __syncthreads();
  for (int k = 0; k < w; ++k)
    if (i < w) Inv[(int64_t)k * ldi + i] = (i >= k) ? Ls[i * 65 + k] : 0.0;
}

hipError_t launch_potrf_small(double* A, int64_t lda, int w, double* Inv, int64_t ldi,
                              unsigned long long* info, int64_t row0, hipStream_t s) {
  if (w < 1 || w > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(potrf_small_kernel, dim3(1), dim3(64), 0, s, A, lda, w, Inv, ldi, info, row0);
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

// y[0:m] = beta * y + alpha * A[0:m, 0:k] x   (A column-major).  Workgroup
// of 64 rows; its sixteen waves take a sixteenth of the columns each, eight
// loads in flight per lane, and add their sums through LDS.
constexpr int kGemvWaves = 16;
__global__ void __launch_bounds__(64 * kGemvWaves) gemv_n_kernel(const double* __restrict__ A, int64_t lda, int64_t m,
                                                                 int64_t k, const double* __restrict__ x,
                                                                 double alpha, double beta, double* __restrict__ y) {
  __shared__ double red[kGemvWaves][64];
  const int rl = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * 64 + rl;
  const int64_t ic = i < m ? i : m - 1;   // rows past m read row m - 1 (not stored)
  const int64_t kq = (k + kGemvWaves - 1) / kGemvWaves;
  const int64_t c0 = g * kq, c1 = (c0 + kq < k) ? c0 + kq : k;
  double acc[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) acc[u] = 0.0;
  int64_t c = c0;
  for (; c + 8 <= c1; c += 8) {
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u] += A[(c + u) * lda + ic] * x[c + u];
  }
  for (; c < c1; ++c) acc[0] += A[c * lda + ic] * x[c];
  red[g][rl] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  __syncthreads();
  if (g == 0 && i < m) {
    double v = 0.0;
#pragma unroll
    for (int q = 0; q < kGemvWaves; ++q) v += red[q][rl];
    y[i] = (beta == 0.0 ? 0.0 : beta * y[i]) + alpha * v;
  }
}

hipError_t launch_gemv_n(const double* A, int64_t lda, int64_t m, int64_t k, const double* x, double alpha,
                         double beta, double* y, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(gemv_n_kernel, dim3((unsigned)((m + 63) / 64)), dim3(64 * kGemvWaves), 0, s, A, lda, m, k, x,
                     alpha, beta, y);
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

// *acc += sum of (A - B)^2 over an m x ncol block (B null: sum of A^2), both
// column-major.  Grid-stride over the elements, one atomic add per workgroup.
__global__ void __launch_bounds__(256) sqdiff_acc_kernel(const double* __restrict__ A, int64_t lda,
                                                         const double* __restrict__ B, int64_t ldb, int64_t m,
                                                         int64_t ncol, double* acc) {
  __shared__ double part[4];
  const int64_t tot = m * ncol;
  double s = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (int64_t)gridDim.x * 256) {
    const int64_t c = e / m, r = e - c * m;
    double d = A[c * lda + r];
    if (B) d -= B[c * ldb + r];
    s += d * d;
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(acc, (part[0] + part[1]) + (part[2] + part[3]));
}

hipError_t launch_sqdiff_acc(const double* A, int64_t lda, const double* B, int64_t ldb, int64_t m, int64_t ncol,
                             double* acc, hipStream_t s) {
  if (m <= 0 || ncol <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>(128, (m * ncol + 255) / 256);
  hipLaunchKernelGGL(sqdiff_acc_kernel, dim3((unsigned)blocks), dim3(256), 0, s, A, lda, B, ldb, m, ncol, acc);
  return hipGetLastError();
}

hipError_t launch_dot(const double* a, const double* b, int64_t m, double* out, hipStream_t s) {
  hipLaunchKernelGGL(dot_kernel, dim3(1), dim3(256), 0, s, a, b, m, out);
  return hipGetLastError();
}

// Copy n ints (and optionally one 64-bit word) into fine-grained host memory,
// then store seq to *flag with release semantics at system scope: a host that
// reads *flag == seq (acquire) then sees the copied values.  One workgroup.
__global__ void __launch_bounds__(256) publish_kernel(const int* __restrict__ src, int n, int* dst,
                                                      const unsigned long long* __restrict__ w_src,
                                                      unsigned long long* w_dst, unsigned* flag, unsigned seq) {
  for (int i = threadIdx.x; i < n; i += 256) dst[i] = src[i];
  if (threadIdx.x == 0 && w_src) *w_dst = *w_src;
  __threadfence_system();   // each thread's stores complete at system scope before the flag
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(flag, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

hipError_t launch_publish(const int* src, int n, int* dst, const unsigned long long* w_src, unsigned long long* w_dst,
                          unsigned* flag, unsigned seq, hipStream_t s) {
  if (n < 0 || (n > 0 && (!src || !dst)) || !flag || (w_src && !w_dst)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(publish_kernel, dim3(1), dim3(256), 0, s, src, n, dst, w_src, w_dst, flag, seq);
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
