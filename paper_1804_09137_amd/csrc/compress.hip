// Tile compression kernels (Section V: each off-diagonal tile is replaced by
// U V^T, keeping what exceeds an absolute accuracy threshold).
//
// Method used on the GPU (the paper allows SVD, randomized SVD or ACA):
//   1. sketch       Y = C Omega            (MFMA GEMM, Omega Gaussian)
//   2. range        Y Pi = Q1 R1 by column-pivoted Householder QR, stopped
//                   when the Frobenius norm of the unreduced block of Y is
//                   below a small fraction of the threshold
//   3. project      B^T = C^T Q1           (MFMA GEMM)
//   4. truncate     B^T Pi2 = Q2 R2 by column-pivoted Householder QR, stopped
//                   when ||R2[k:, k:]||_F <= threshold
//   5. assemble     U = Q1 Pi2 R2[:k, :]^T, V = Q2[:, :k]
// so ||C - U V^T||_2 <= ||(I - Q1 Q1^T) C||_2 + ||R2[k:, k:]||_F.
//
// qrcp_kernel is one 1024-thread workgroup per matrix; the matrix stays in
// global memory (L2-resident), each of the 16 waves owns a set of columns and
// keeps its column slice in registers during a Householder application.
#include "kernels.h"
#include "compress.h"

namespace tlrk {

constexpr int kQrThreads = 1024;
constexpr int kQrWaves = kQrThreads / 64;

__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__global__ void __launch_bounds__(kQrThreads) qrcp_kernel(const QrcpTask* __restrict__ tasks) {
  const QrcpTask tk = tasks[blockIdx.x];
  __shared__ double nrm[kQrMaxCols];
  __shared__ double tau[kQrMaxCols];
  __shared__ int perm[kQrMaxCols];
  __shared__ double vs[kQrMaxRows];
  __shared__ double red[kQrWaves];
  __shared__ int sh_piv, sh_stop;
  __shared__ double sh_beta, sh_tau, sh_scale;

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int m = tk.m, q = tk.q;
  double* Y = tk.Y;
  const int64_t ld = tk.ldy;
  if (m <= 0 || q <= 0) {
    if (tid == 0) {
      if (tk.rank) *tk.rank = 0;
      if (tk.flag) *tk.flag = 0;
    }
    return;
  }

  for (int c = wv; c < q; c += kQrWaves) {
    double s = 0.0;
    for (int r = lane; r < m; r += 64) {
      const double v = Y[c * ld + r];
      s += v * v;
    }
    s = wave_sum(s);
    if (lane == 0) nrm[c] = s;
  }
  for (int c = tid; c < q; c += kQrThreads) perm[c] = c;
  __syncthreads();

  const int tmax = m < q ? m : q;
  const double tol2 = tk.tol * tk.tol;
  int t = 0;
  for (; t < tmax; ++t) {
    if (wv == 0) {
      double s = 0.0, best = -1.0;
      int bi = t;
      for (int c = t + lane; c < q; c += 64) {
        const double v = nrm[c];
        s += v;
        if (v > best) { best = v; bi = c; }
      }
      s = wave_sum(s);
      for (int off = 32; off > 0; off >>= 1) {
        const double ob = __shfl_xor(best, off, 64);
        const int oi = __shfl_xor(bi, off, 64);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      if (lane == 0) {
        sh_stop = (s <= tol2 || t >= tk.max_rank) ? 1 : 0;
        sh_piv = bi;
      }
    }
    __syncthreads();
    if (sh_stop) break;
    const int p = sh_piv;
    if (p != t) {
      for (int r = tid; r < m; r += kQrThreads) {
        const double a = Y[(int64_t)t * ld + r];
        Y[(int64_t)t * ld + r] = Y[(int64_t)p * ld + r];
        Y[(int64_t)p * ld + r] = a;
      }
      if (tid == 0) {
        const double a = nrm[t]; nrm[t] = nrm[p]; nrm[p] = a;
        const int b = perm[t]; perm[t] = perm[p]; perm[p] = b;
      }
    }
    __syncthreads();
    // Householder vector of column t (rows t..m-1)
    {
      double s = 0.0;
      for (int r = t + 1 + tid; r < m; r += kQrThreads) {
        const double v = Y[(int64_t)t * ld + r];
        s += v * v;
      }
      s = wave_sum(s);
      if (lane == 0) red[wv] = s;
      __syncthreads();
      if (tid == 0) {
        double sig = 0.0;
        for (int w = 0; w < kQrWaves; ++w) sig += red[w];
        const double alpha = Y[(int64_t)t * ld + t];
        if (sig == 0.0) {
          sh_tau = 0.0; sh_beta = alpha; sh_scale = 0.0;
        } else {
          const double nx = sqrt(alpha * alpha + sig);
          const double beta = alpha >= 0.0 ? -nx : nx;
          sh_tau = (beta - alpha) / beta;
          sh_scale = 1.0 / (alpha - beta);
          sh_beta = beta;
        }
        tau[t] = sh_tau;
      }
      __syncthreads();
      const double sc = sh_scale;
      for (int r = t + tid; r < m; r += kQrThreads) {
        double v;
        if (r == t) {
          v = 1.0;
          Y[(int64_t)t * ld + t] = sh_beta;
        } else {
          v = Y[(int64_t)t * ld + r] * sc;
          Y[(int64_t)t * ld + r] = v;
        }
        vs[r] = v;
      }
      __syncthreads();
    }
    // apply H_t to columns t+1..q-1 and refresh their norms over rows > t
    const double ta = sh_tau;
    for (int c = t + 1 + wv; c < q; c += kQrWaves) {
      double* col = Y + (int64_t)c * ld;
      double yv[kQrMaxRows / 64];
      double w = 0.0;
#pragma unroll
      for (int i = 0; i < kQrMaxRows / 64; ++i) {
        const int r = t + lane + 64 * i;
        yv[i] = (r < m) ? col[r] : 0.0;
        if (r < m) w += vs[r] * yv[i];
      }
      w = wave_sum(w) * ta;
      double s = 0.0;
#pragma unroll
      for (int i = 0; i < kQrMaxRows / 64; ++i) {
        const int r = t + lane + 64 * i;
        if (r < m) {
          const double nv = yv[i] - w * vs[r];
          col[r] = nv;
          if (r > t) s += nv * nv;
        }
      }
      s = wave_sum(s);
      if (lane == 0) nrm[c] = s;
    }
    __syncthreads();
  }
  const int rank = t;
  if (tid == 0) {
    if (tk.rank) *tk.rank = rank;
    if (tk.flag) *tk.flag = (q - rank < tk.min_tail) ? 1 : 0;
  }

  // Z[perm[c], r] = R[r, c] for r < rank, c < q
  if (tk.Z) {
    for (int e = tid; e < q * rank; e += kQrThreads) {
      const int c = e % q, r = e / q;
      tk.Z[(int64_t)r * tk.ldz + perm[c]] = (c >= r) ? Y[(int64_t)c * ld + r] : 0.0;
    }
  }
  if (!tk.Q) return;
  // explicit Q = H_0 ... H_{rank-1} [I; 0]  (m x rank)
  double* Q = tk.Q;
  const int64_t ldq = tk.ldq;
  for (int e = tid; e < m * rank; e += kQrThreads) {
    const int r = e % m, c = e / m;
    Q[(int64_t)c * ldq + r] = (r == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int s = rank - 1; s >= 0; --s) {
    for (int r = s + tid; r < m; r += kQrThreads) vs[r] = (r == s) ? 1.0 : Y[(int64_t)s * ld + r];
    __syncthreads();
    const double ta = tau[s];
    for (int c = s + wv; c < rank; c += kQrWaves) {
      double* col = Q + (int64_t)c * ldq;
      double yv[kQrMaxRows / 64];
      double w = 0.0;
#pragma unroll
      for (int i = 0; i < kQrMaxRows / 64; ++i) {
        const int r = s + lane + 64 * i;
        yv[i] = (r < m) ? col[r] : 0.0;
        if (r < m) w += vs[r] * yv[i];
      }
      w = wave_sum(w) * ta;
#pragma unroll
      for (int i = 0; i < kQrMaxRows / 64; ++i) {
        const int r = s + lane + 64 * i;
        if (r < m) col[r] = yv[i] - w * vs[r];
      }
    }
    __syncthreads();
  }
}

hipError_t launch_qrcp(const QrcpTask* d_tasks, int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(qrcp_kernel, dim3((unsigned)count), dim3(kQrThreads), 0, s, d_tasks);
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
