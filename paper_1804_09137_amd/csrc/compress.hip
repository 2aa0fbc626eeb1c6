// Compression helpers (Section V: each off-diagonal tile is replaced by
// U V^T, keeping what exceeds an absolute accuracy threshold).  The pipeline
// itself (sketch, blocked Householder QR, range rank, projection, truncation)
// is described in hqr.hip; this file holds:
//   * qrcp_kernel: column-pivoted Householder QR of a matrix in global memory
//     (L2-resident), one 512-thread workgroup per matrix, stopped when the
//     Frobenius norm of the unreduced block is <= tol or at max_rank; used for
//     the small truncation factors too large for the register-resident
//     qrcp_reg_kernel.  Each of the 8 waves owns a set of columns and keeps
//     two column slices in registers during a Householder application.
//   * the Gaussian sketch matrix (Philox4x32-10 + Box-Muller);
//   * a batched block copy.
#include "kernels.h"
#include "compress.h"
#include "wave.h"

namespace tlrk {

constexpr int kQrThreads = 512;
constexpr int kQrWaves = kQrThreads / 64;


// Column-pivoted Householder QR, one workgroup per matrix.  Columns are never
// moved: piv[t] records the physical column chosen at step t and step_of[]
// its inverse.  Each step: (1) the pivot column's reflector (block reduction),
// (2) every live column is reflected and its norm over rows > t recomputed
// exactly; the per-wave partial sums and maxima of those norms feed the next
// step's stopping test and pivot choice.  Three barriers per step.
// RPL: rows per lane (m <= 64 RPL); CB: columns a wave reflects at once (their
// loads are in flight together: the step's latency is q / (8 CB) round trips).
template <int RPL, int CB>
__global__ void __launch_bounds__(kQrThreads) qrcp_kernel(const QrcpTask* __restrict__ tasks) {
  const QrcpTask tk = tasks[blockIdx.x];
  __shared__ double nrm[kQrMaxCols];
  __shared__ double tau[kQrMaxCols];
  __shared__ int piv[kQrMaxCols];
  __shared__ int step_of[kQrMaxCols];
  __shared__ double vs[kQrMaxRows];
  __shared__ double red[kQrWaves];
  __shared__ double wsum[kQrWaves], wmax[kQrWaves];
  __shared__ int widx[kQrWaves];
  __shared__ double sh_alpha;

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int m = tk.m, q = tk.q;
  double* Y = tk.Y;
  const int64_t ld = tk.ldy;
  if (m <= 0 || q <= 0 || m > 64 * RPL || q > kQrMaxCols) {
    if (tid == 0) {
      if (tk.rank) *tk.rank = 0;
      if (tk.flag) *tk.flag = (m > 0 && q > 0) ? 1 : 0;
    }
    return;
  }

  // initial norms and per-wave partials
  {
    double ls = 0.0, lm = -1.0;
    int li = 0x7fffffff;
    for (int c = wv; c < q; c += kQrWaves) {
      double sacc = 0.0;
      for (int r = lane; r < m; r += 64) {
        const double v = Y[(int64_t)c * ld + r];
        sacc += v * v;
      }
      sacc = wave::sum(sacc);
      if (lane == 0) nrm[c] = sacc;
      ls += sacc;
      if (sacc > lm || (sacc == lm && c < li)) { lm = sacc; li = c; }
    }
    if (lane == 0) { wsum[wv] = ls; wmax[wv] = lm; widx[wv] = li; }
    for (int c = tid; c < q; c += kQrThreads) step_of[c] = 0x7fffffff;
  }
  __syncthreads();

  const int tmax = m < q ? m : q;
  const double tol2 = tk.tol * tk.tol;
  int t = 0;
  for (; t < tmax; ++t) {
    // every thread reduces the wave partials identically
    double total = 0.0, best = -1.0;
    int p = 0x7fffffff;
#pragma unroll
    for (int w = 0; w < kQrWaves; ++w) {
      total += wsum[w];
      if (wmax[w] > best || (wmax[w] == best && widx[w] < p)) { best = wmax[w]; p = widx[w]; }
    }
    if (total <= tol2 || t >= tk.max_rank || p >= q) break;
    // reflector of column p, rows t..m-1 (two rows per thread: m <= 1024)
    double* colp = Y + (int64_t)p * ld;
    const int r = t + tid;
    const int r2 = r + kQrThreads;
    double x = 0.0, x2 = 0.0;
    if (r < m) x = colp[r];
    if (r2 < m) x2 = colp[r2];
    if (r == t) sh_alpha = x;
    double sp = (r > t && r < m) ? x * x : 0.0;
    sp += (r2 < m) ? x2 * x2 : 0.0;
    sp = wave::sum(sp);
    if (lane == 0) red[wv] = sp;
    if (tid == 0) { piv[t] = p; step_of[p] = t; }
    __syncthreads();
    double sig = 0.0;
#pragma unroll
    for (int w = 0; w < kQrWaves; ++w) sig += red[w];
    const double alpha = sh_alpha;
    double ta, beta, sc;
    if (sig == 0.0) {
      ta = 0.0; beta = alpha; sc = 0.0;
    } else {
      const double nx = sqrt(alpha * alpha + sig);
      beta = alpha >= 0.0 ? -nx : nx;
      ta = (beta - alpha) / beta;
      sc = 1.0 / (alpha - beta);
    }
    if (r < m) {
      if (r == t) { vs[r] = 1.0; colp[r] = beta; }
      else { const double v = x * sc; vs[r] = v; colp[r] = v; }
    }
    if (r2 < m) { const double v = x2 * sc; vs[r2] = v; colp[r2] = v; }
    if (tid == 0) tau[t] = ta;
    __syncthreads();
    // reflect the live columns, CB per wave at a time
    double vv[RPL];
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      const int rr = t + lane + 64 * i;
      vv[i] = rr < m ? vs[rr] : 0.0;
    }
    double ls = 0.0, lm = -1.0;
    int li = 0x7fffffff;
    for (int c0 = wv; c0 < q; c0 += CB * kQrWaves) {
      double v[CB][RPL];
      bool act[CB];
      double w[CB];
#pragma unroll
      for (int b = 0; b < CB; ++b) {
        const int c = c0 + b * kQrWaves;
        act[b] = (c < q) && (step_of[c] > t) && (c != p);
        const double* yc = Y + (int64_t)(act[b] ? c : c0) * ld;
        w[b] = 0.0;
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
          const int rr = t + lane + 64 * i;
          v[b][i] = (act[b] && rr < m) ? yc[rr] : 0.0;
          w[b] += vv[i] * v[b][i];
        }
      }
#pragma unroll
      for (int b = 0; b < CB; ++b) w[b] = wave::sum(w[b]) * ta;
#pragma unroll
      for (int b = 0; b < CB; ++b) {
        const int c = c0 + b * kQrWaves;
        double* yc = Y + (int64_t)(act[b] ? c : c0) * ld;
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
          const int rr = t + lane + 64 * i;
          if (rr < m) {
            const double nv = v[b][i] - w[b] * vv[i];
            if (act[b]) yc[rr] = nv;
            if (rr > t) s += nv * nv;
          }
        }
        s = wave::sum(s);
        if (act[b]) {
          if (lane == 0) nrm[c] = s;
          ls += s;
          if (s > lm || (s == lm && c < li)) { lm = s; li = c; }
        }
      }
    }
    if (lane == 0) { wsum[wv] = ls; wmax[wv] = lm; widx[wv] = li; }
    __syncthreads();
  }
  const int rank = t;
  if (tid == 0) {
    if (tk.rank) *tk.rank = rank;
    if (tk.flag) *tk.flag = (q - rank < tk.min_tail) ? 1 : 0;
  }

  // Z[c, r] = R[r, step_of[c]] for r < rank: column c holds its R entries in
  // rows <= step_of[c] (all rows < rank if c was never chosen)
  if (tk.Z) {
    for (int e = tid; e < q * rank; e += kQrThreads) {
      const int c = e % q, rr = e / q;
      tk.Z[(int64_t)rr * tk.ldz + c] = (step_of[c] >= rr) ? Y[(int64_t)c * ld + rr] : 0.0;
    }
  }
  if (!tk.Q) return;
  // explicit Q = H_0 ... H_{rank-1} [I; 0]  (m x rank); reflector s lives in
  // column piv[s], rows > s
  double* Q = tk.Q;
  const int64_t ldq = tk.ldq;
  for (int e = tid; e < m * rank; e += kQrThreads) {
    const int rr = e % m, c = e / m;
    Q[(int64_t)c * ldq + rr] = (rr == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int st = rank - 1; st >= 0; --st) {
    const double* vcol = Y + (int64_t)piv[st] * ld;
    for (int rr = st + tid; rr < m; rr += kQrThreads) vs[rr] = (rr == st) ? 1.0 : vcol[rr];
    __syncthreads();
    const double ta = tau[st];
    double vv[RPL];
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      const int rr = st + lane + 64 * i;
      vv[i] = rr < m ? vs[rr] : 0.0;
    }
    for (int c0 = st + wv; c0 < rank; c0 += CB * kQrWaves) {
      double v[CB][RPL];
      double w[CB];
#pragma unroll
      for (int b = 0; b < CB; ++b) {
        const int c = c0 + b * kQrWaves;
        const bool a = c < rank;
        const double* yc = Q + (int64_t)(a ? c : c0) * ldq;
        w[b] = 0.0;
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
          const int rr = st + lane + 64 * i;
          v[b][i] = (a && rr < m) ? yc[rr] : 0.0;
          w[b] += vv[i] * v[b][i];
        }
      }
#pragma unroll
      for (int b = 0; b < CB; ++b) w[b] = wave::sum(w[b]) * ta;
#pragma unroll
      for (int b = 0; b < CB; ++b) {
        const int c = c0 + b * kQrWaves;
        if (c >= rank) continue;
        double* yc = Q + (int64_t)c * ldq;
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
          const int rr = st + lane + 64 * i;
          if (rr < m) yc[rr] = v[b][i] - w[b] * vv[i];
        }
      }
    }
    __syncthreads();
  }
}

// Tasks are launched with the smallest row capacity that fits the largest m.
hipError_t launch_qrcp(const QrcpTask* d_tasks, int count, hipStream_t s, int max_m) {
  if (count <= 0) return hipSuccess;
  if (max_m <= 256)
    hipLaunchKernelGGL((qrcp_kernel<4, 8>), dim3((unsigned)count), dim3(kQrThreads), 0, s, d_tasks);
  else if (max_m <= 512)
    hipLaunchKernelGGL((qrcp_kernel<8, 6>), dim3((unsigned)count), dim3(kQrThreads), 0, s, d_tasks);
  else
    hipLaunchKernelGGL((qrcp_kernel<16, 3>), dim3((unsigned)count), dim3(kQrThreads), 0, s, d_tasks);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Gaussian sketch matrix: Philox4x32-10 counter-based generator (Salmon,
// Moraes, Dror, Shaw, SC'11) keyed by the seed, counter = element index,
// mapped to N(0,1) by the Box-Muller transform.
// ---------------------------------------------------------------------------
__device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)M0 * c[0];
    const uint64_t p1 = (uint64_t)M1 * c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k0;
    const uint32_t n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
    k0 += W0; k1 += W1;
  }
}

__global__ void gaussian_kernel(double* out, int64_t count, uint32_t seed) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i * 2 >= count) return;
  uint32_t c[4] = {(uint32_t)i, (uint32_t)(i >> 32), 0x5EEDu, 0u};
  philox4x32_10(c, seed, 0x6A09E667u);
  const double u1 = ((double)c[0] + 1.0) * (1.0 / 4294967297.0);   // (0, 1]
  const double u2 = (double)c[1] * (1.0 / 4294967296.0);           // [0, 1)
  const double rad = sqrt(-2.0 * log(u1));
  double sn, cs;
  sincos(6.283185307179586 * u2, &sn, &cs);
  out[2 * i] = rad * cs;
  if (2 * i + 1 < count) out[2 * i + 1] = rad * sn;
}

hipError_t launch_gaussian(double* out, int64_t count, uint32_t seed, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const int64_t pairs = (count + 1) / 2;
  hipLaunchKernelGGL(gaussian_kernel, dim3((unsigned)((pairs + 255) / 256)), dim3(256), 0, s, out, count, seed);
  return hipGetLastError();
}

// Batched column-block copy: for task b, copy rows [0, m_b) x cols [0, k_b)
// from src + soff[b] (ld sld) to dst + doff[b] (ld dld); grid.y = batch.
__global__ void batched_copy_kernel(const double* __restrict__ src, int64_t sld, const int64_t* __restrict__ soff,
                                    double* __restrict__ dst, int64_t dld, const int64_t* __restrict__ doff,
                                    const int* __restrict__ mrows, const int* __restrict__ kcols, int64_t mmax) {
  const int b = blockIdx.y;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int m = mrows[b], k = kcols[b];
  if (e >= (int64_t)m * k) return;
  const int64_t r = e % m, c = e / m;
  dst[doff[b] + c * dld + r] = src[soff[b] + c * sld + r];
  (void)mmax;
}

hipError_t launch_batched_copy(const double* src, int64_t sld, const int64_t* soff, double* dst, int64_t dld,
                               const int64_t* doff, const int* mrows, const int* kcols, int64_t max_elems,
                               int count, hipStream_t s) {
  if (count <= 0 || max_elems <= 0) return hipSuccess;
  hipLaunchKernelGGL(batched_copy_kernel, dim3((unsigned)((max_elems + 255) / 256), (unsigned)count), dim3(256), 0,
                     s, src, sld, soff, dst, dld, doff, mrows, kcols, max_elems);
  return hipGetLastError();
}

}  // namespace tlrk
