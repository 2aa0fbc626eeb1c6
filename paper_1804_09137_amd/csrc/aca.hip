// Adaptive cross approximation (ACA) with partial pivoting of Matérn tiles,
// fused with their generation: a tile A (m x n, rows r0.., columns c0.. of
// Sigma, Eq. (MaternCov)) is never formed; each step generates one row and one
// column of it (Section V lists ACA among the compressions).
//
// Step k (Bebendorf, Numer. Math. 86 (2000); partial pivoting):
//   row      r = A[i*, :] - sum_{l<k} U[i*, l] V[:, l]^T, pivot column j* = argmax |r_j| (unused columns)
//   v_k      = r / r[j*]
//   column   u_k = A[:, j*] - sum_{l<k} U[:, l] V[j*, l]
//   next row i* = argmax |u_k,i| over unused rows
// so that A ~ U V^T.  The stop is absolute (the threshold of Section V is):
// two consecutive terms with ||u_k|| ||v_k|| <= tau (both then dropped), a
// zero residual on every row tried, or k = kmax (then *rank = kmax + 1: the
// tile needs more).  One 256-thread workgroup per tile; the current row and
// column live in LDS.
#include "kernels.h"
#include "matern.h"
#include "aca.h"

namespace tlrk {

namespace {

constexpr int kAcaThreads = 256;
constexpr int kAcaMaxDim = 1024;

// argmax of |val| over the block (ties: the smaller index); returns (index, value)
__device__ inline void block_argmax(double av, int idx, double* sv, int* si, double& bv, int& bi) {
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_down(av, off, 64);
    const int oi = __shfl_down(idx, off, 64);
    if (ov > av || (ov == av && oi < idx)) {
      av = ov;
      idx = oi;
    }
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sv[w] = av;
    si[w] = idx;
  }
  __syncthreads();
  bv = sv[0];
  bi = si[0];
  for (int q = 1; q < kAcaThreads / 64; ++q)
    if (sv[q] > bv || (sv[q] == bv && si[q] < bi)) {
      bv = sv[q];
      bi = si[q];
    }
  __syncthreads();
}

__device__ inline double block_sum(double v, double* sv) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if ((threadIdx.x & 63) == 0) sv[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int q = 0; q < kAcaThreads / 64; ++q) s += sv[q];
  __syncthreads();
  return s;
}

}  // namespace

__global__ void __launch_bounds__(kAcaThreads) aca_kernel(MaternParams p, const double* __restrict__ x,
                                                          const double* __restrict__ y, const AcaTask* tasks,
                                                          int kmax, double tau) {
  __shared__ double rowb[kAcaMaxDim], colb[kAcaMaxDim];
  __shared__ unsigned char used_r[kAcaMaxDim], used_c[kAcaMaxDim];
  __shared__ double sv[kAcaThreads / 64];
  __shared__ int si[kAcaThreads / 64];
  const AcaTask t = tasks[blockIdx.x];
  const int m = t.m, n = t.n, tid = threadIdx.x;
  for (int i = tid; i < kAcaMaxDim; i += kAcaThreads) {
    used_r[i] = 0;
    used_c[i] = 0;
  }
  __syncthreads();
  int ist = 0, k = 0, small = 0, tried = 0;
  while (k < kmax) {
    // residual row i* (U row entries are read from global: U[ist + l ld])
    for (int j = tid; j < n; j += kAcaThreads) {
      double c, d;
      matern_eval<false>(p, loc_dist(p, x, y, t.r0 + ist, t.c0 + j), c, d);
      for (int l = 0; l < k; ++l) c -= t.U[ist + l * t.ld] * t.V[j + l * t.ld];
      rowb[j] = c;
    }
    __syncthreads();
    double best = -1.0;
    int bj = 0x7fffffff;
    for (int j = tid; j < n; j += kAcaThreads) {
      const double a = used_c[j] ? -1.0 : fabs(rowb[j]);
      if (a > best || (a == best && j < bj)) {
        best = a;
        bj = j;
      }
    }
    double pv;
    int jst;
    block_argmax(best, bj, sv, si, pv, jst);
    if (!(pv > 0.0)) {
      // this row's residual vanishes: try the next unused row
      if (tid == 0) used_r[ist] = 1;
      __syncthreads();
      if (++tried >= m) break;
      int nx = 0x7fffffff;
      for (int i = tid; i < m; i += kAcaThreads)
        if (!used_r[i] && i < nx) nx = i;
      double dummy;
      int nxt;
      block_argmax(0.0, nx, sv, si, dummy, nxt);
      if (nxt >= m) break;
      ist = nxt;
      continue;
    }
    const double piv = rowb[jst];
    // v_k = row / pivot
    double vv = 0.0;
    for (int j = tid; j < n; j += kAcaThreads) {
      const double v = rowb[j] / piv;
      t.V[j + k * t.ld] = v;
      vv += v * v;
    }
    // u_k = residual column j*
    double uu = 0.0;
    for (int i = tid; i < m; i += kAcaThreads) {
      double c, d;
      matern_eval<false>(p, loc_dist(p, x, y, t.r0 + i, t.c0 + jst), c, d);
      for (int l = 0; l < k; ++l) c -= t.U[i + l * t.ld] * t.V[jst + l * t.ld];
      colb[i] = c;
      t.U[i + k * t.ld] = c;
      uu += c * c;
    }
    if (tid == 0) {
      used_r[ist] = 1;
      used_c[jst] = 1;
    }
    const double su = block_sum(uu, sv);
    const double svv = block_sum(vv, sv);
    ++k;
    tried = 0;
    small = (sqrt(su) * sqrt(svv) <= tau) ? small + 1 : 0;
    if (small >= 2) break;
    double bu = -1.0;
    int bi = 0x7fffffff;
    for (int i = tid; i < m; i += kAcaThreads) {
      const double a = used_r[i] ? -1.0 : fabs(colb[i]);
      if (a > bu || (a == bu && i < bi)) {
        bu = a;
        bi = i;
      }
    }
    double dummy;
    int nxt;
    block_argmax(bu, bi, sv, si, dummy, nxt);
    if (nxt >= m || dummy < 0.0) break;   // every row used
    ist = nxt;
  }
  // the trailing terms below tau are dropped (at most two, each of spectral
  // norm ||u|| ||v|| <= tau)
  if (tid == 0) *t.rank = (k >= kmax && small < 2) ? kmax + 1 : k - small;
}

hipError_t launch_aca(const MaternParams& p, const double* x, const double* y, const AcaTask* d_tasks, int count,
                      int kmax, double tau, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(aca_kernel, dim3((unsigned)count), dim3(kAcaThreads), 0, s, p, x, y, d_tasks, kmax, tau);
  return hipGetLastError();
}

}  // namespace tlrk
