// Triangular solves over a TLR factor (Section III: the likelihood needs
// z^T Sigma^{-1} z = ||L^{-1} z||^2; the score needs a = L^{-T} L^{-1} z).
//
// lowrank_apply_kernel: workgroup (tile, y) computes t = B^T v (k dots of
// length nb, 16 at a time per wave with one transposed butterfly) and then
// out -= A t for rows [256 y, 256 y + 256) of its tile, one row per thread.
#include "kernels.h"
#include "solve.h"
#include "wave.h"

namespace tlrk {

constexpr int kLrMaxRank = 1024;

__global__ void __launch_bounds__(256) lowrank_apply_kernel(LowRankApply a) {
  __shared__ double t[kLrMaxRank];
  const int b = blockIdx.x;
  int ti, tj;      // tile (ti, tj), ti > tj, of the factor
  int64_t src0, dst0;
  int msrc, mdst;
  const double* Bm;
  const double* Am;
  if (a.forward) {  // column a.fixed: tiles (fixed + 1 + b, fixed); v = y_fixed, out = z_i
    ti = a.fixed + 1 + b;
    tj = a.fixed;
  } else {          // row a.fixed: tiles (fixed, b); v = alpha_fixed, out = r_b
    ti = a.fixed;
    tj = b;
  }
  const int64_t id = (int64_t)ti * a.nt + tj;
  const int k = a.ranks[id];
  if (k <= 0) return;
  const int mi = (ti == a.nt - 1) ? (int)(a.n - (int64_t)ti * a.nb) : a.nb;
  const int mj = (tj == a.nt - 1) ? (int)(a.n - (int64_t)tj * a.nb) : a.nb;
  if (a.forward) {  // t = V^T y_j, z_i -= U t
    Bm = a.arena + a.voff[id];
    Am = a.arena + a.uoff[id];
    src0 = (int64_t)tj * a.nb; msrc = mj;
    dst0 = (int64_t)ti * a.nb; mdst = mi;
  } else {          // t = U^T alpha_i, r_j -= V t
    Bm = a.arena + a.uoff[id];
    Am = a.arena + a.voff[id];
    src0 = (int64_t)ti * a.nb; msrc = mi;
    dst0 = (int64_t)tj * a.nb; mdst = mj;
  }
  const int r0 = blockIdx.y * 256;
  if (r0 >= mdst) return;   // uniform over the workgroup
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int c0 = 16 * wv; c0 < k; c0 += 64) {
    double part[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) part[q] = 0.0;
    // columns past k read column k - 1 (in bounds, not stored): no branches
    // around the loads, sixteen in flight per lane
    const double* bq[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) bq[q] = Bm + (int64_t)(c0 + q < k ? c0 + q : k - 1) * a.nb;
#pragma unroll 4
    for (int r = lane; r < msrc; r += 64) {
      const double vr = a.v[src0 + r];
#pragma unroll
      for (int q = 0; q < 16; ++q) part[q] += bq[q][r] * vr;
    }
    const double tot = wave::bfly<16>(part, lane);
    const int q = (lane >> 2) & 15;
    if ((lane & 3) == 0 && c0 + q < k) t[c0 + q] = tot;
  }
  __syncthreads();
  const int r = r0 + threadIdx.x;
  if (r < mdst) {
    double acc[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) acc[u] = 0.0;
    int c = 0;
    for (; c + 16 <= k; c += 16) {
#pragma unroll
      for (int u = 0; u < 16; ++u) acc[u] += Am[(int64_t)(c + u) * a.nb + r] * t[c + u];
    }
    for (; c < k; ++c) acc[0] += Am[(int64_t)c * a.nb + r] * t[c];
#pragma unroll
    for (int u = 8; u > 0; u >>= 1)
#pragma unroll
      for (int v = 0; v < u; ++v) acc[v] += acc[v + u];
    const double sum = acc[0];
    // the tiles of one launch write disjoint destination rows
    a.out[dst0 + r] += a.scale * sum;
  }
}

hipError_t launch_lowrank_apply(const LowRankApply& a, int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(lowrank_apply_kernel, dim3((unsigned)count, (unsigned)((a.nb + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace tlrk
