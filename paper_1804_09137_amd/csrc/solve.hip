// Triangular solves over a TLR factor (Section III: the likelihood needs
// z^T Sigma^{-1} z = ||L^{-1} z||^2; the score needs a = L^{-T} L^{-1} z).
//
// Low-rank apply of one column (forward) or row (backward) of tiles: for
// each tile, t = B^T v (k dots of length nb), then out -= A t.  Two launches,
// so that both halves spread over many workgroups (a single workgroup per tile
// is bound by the latency of its chain of loads):
//   lr_dots_kernel:   workgroup (tile, g) takes columns [16 g, 16 g + 16) of B;
//                     its four waves split the rows, each lane sixteen running
//                     dots, one transposed butterfly per wave, LDS across waves;
//   lr_update_kernel: workgroup (tile, y) takes rows [256 y, 256 y + 256) of
//                     out, one row per thread, t staged in LDS.
#include "kernels.h"
#include "solve.h"
#include "wave.h"

namespace tlrk {

struct LrTile {
  int ti, tj, k, msrc, mdst;
  int64_t src0, dst0;
  const double* Bm;
  const double* Am;
};

__device__ inline LrTile lr_tile(const LowRankApply& a, int b) {
  LrTile t;
  if (a.forward) {  // column a.fixed: tiles (fixed + 1 + b, fixed); v = y_fixed, out = z_i
    t.ti = a.fixed + 1 + b;
    t.tj = a.fixed;
  } else {          // row a.fixed: tiles (fixed, b); v = alpha_fixed, out = r_b
    t.ti = a.fixed;
    t.tj = b;
  }
  const int64_t id = (int64_t)t.ti * a.nt + t.tj;
  t.k = a.ranks[id];
  const int mi = (t.ti == a.nt - 1) ? (int)(a.n - (int64_t)t.ti * a.nb) : a.nb;
  const int mj = (t.tj == a.nt - 1) ? (int)(a.n - (int64_t)t.tj * a.nb) : a.nb;
  if (a.forward) {  // t = V^T y_j, z_i -= U t
    t.Bm = a.arena + a.voff[id];
    t.Am = a.arena + a.uoff[id];
    t.src0 = (int64_t)t.tj * a.nb; t.msrc = mj;
    t.dst0 = (int64_t)t.ti * a.nb; t.mdst = mi;
  } else {          // t = U^T alpha_i, r_j -= V t
    t.Bm = a.arena + a.uoff[id];
    t.Am = a.arena + a.voff[id];
    t.src0 = (int64_t)t.ti * a.nb; t.msrc = mi;
    t.dst0 = (int64_t)t.tj * a.nb; t.mdst = mj;
  }
  return t;
}

__global__ void __launch_bounds__(256) lr_dots_kernel(LowRankApply a) {
  __shared__ double red[4][16];
  const LrTile t = lr_tile(a, blockIdx.x);
  const int c0 = 16 * blockIdx.y;
  if (t.k <= 0 || c0 >= t.k) return;   // uniform over the workgroup
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  // columns past k read column k - 1 (in bounds, not stored)
  const double* bq[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) bq[q] = t.Bm + (int64_t)(c0 + q < t.k ? c0 + q : t.k - 1) * a.nb;
  double part[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) part[q] = 0.0;
#pragma unroll 2
  for (int r = 64 * wv + lane; r < t.msrc; r += 256) {
    const double vr = a.v[t.src0 + r];
#pragma unroll
    for (int q = 0; q < 16; ++q) part[q] += bq[q][r] * vr;
  }
  const double tot = wave::bfly<16>(part, lane);
  if ((lane & 3) == 0) red[wv][(lane >> 2) & 15] = tot;
  __syncthreads();
  if (threadIdx.x < 16) {
    const int q = threadIdx.x;
    if (c0 + q < t.k)
      a.tws[(int64_t)blockIdx.x * kLrMaxRank + c0 + q] = (red[0][q] + red[1][q]) + (red[2][q] + red[3][q]);
  }
}

__global__ void __launch_bounds__(256) lr_update_kernel(LowRankApply a) {
  __shared__ double ts[kLrMaxRank];
  const LrTile t = lr_tile(a, blockIdx.x);
  const int r0 = blockIdx.y * 256;
  if (t.k <= 0 || r0 >= t.mdst) return;   // uniform over the workgroup
  for (int c = threadIdx.x; c < t.k; c += 256) ts[c] = a.tws[(int64_t)blockIdx.x * kLrMaxRank + c];
  __syncthreads();
  const int r = r0 + threadIdx.x;
  if (r < t.mdst) {
    double acc[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) acc[u] = 0.0;
    int c = 0;
    for (; c + 16 <= t.k; c += 16) {
#pragma unroll
      for (int u = 0; u < 16; ++u) acc[u] += t.Am[(int64_t)(c + u) * a.nb + r] * ts[c + u];
    }
    for (; c < t.k; ++c) acc[0] += t.Am[(int64_t)c * a.nb + r] * ts[c];
#pragma unroll
    for (int u = 8; u > 0; u >>= 1)
#pragma unroll
      for (int v = 0; v < u; ++v) acc[v] += acc[v + u];
    // the tiles of one launch write disjoint destination rows
    a.out[t.dst0 + r] += a.scale * acc[0];
  }
}

hipError_t launch_lowrank_apply(const LowRankApply& a, int count, hipStream_t s, int kmax) {
  if (count <= 0) return hipSuccess;
  if (!a.tws || kmax > kLrMaxRank) return hipErrorInvalidValue;
  if (kmax <= 0) return hipSuccess;
  hipLaunchKernelGGL(lr_dots_kernel, dim3((unsigned)count, (unsigned)((kmax + 15) / 16)), dim3(256), 0, s, a);
  hipLaunchKernelGGL(lr_update_kernel, dim3((unsigned)count, (unsigned)((a.nb + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace tlrk
