// Triangular solves over a TLR factor (Section III: the likelihood needs
// z^T Sigma^{-1} z = ||L^{-1} z||^2; the score needs a = L^{-T} L^{-1} z).
//
// lowrank_apply_kernel: one workgroup per tile; computes t = B^T v (k dots of
// length nb, wave reductions into LDS) and then out -= A t.
#include "kernels.h"
#include "solve.h"

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
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int c = wv; c < k; c += 4) {
    double s = 0.0;
    for (int r = lane; r < msrc; r += 64) s += Bm[(int64_t)c * a.nb + r] * a.v[src0 + r];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) t[c] = s;
  }
  __syncthreads();
  for (int r = threadIdx.x; r < mdst; r += 256) {
    double acc = 0.0;
    for (int c = 0; c < k; ++c) acc += Am[(int64_t)c * a.nb + r] * t[c];
    // the tiles of one launch write disjoint destination rows
    a.out[dst0 + r] += a.scale * acc;
  }
}

hipError_t launch_lowrank_apply(const LowRankApply& a, int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(lowrank_apply_kernel, dim3((unsigned)count), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace tlrk
