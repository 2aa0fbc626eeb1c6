// Blocked Householder QR of tall tiles and a register-resident column-pivoted
// QR of the small triangular factors they produce.  Together they replace a
// pivoted QR of the tall sketch (whose every pivot step streams the whole
// matrix) in the randomized compression of Section V:
//
//   Y = C Omega = Q_y R_y              hqr_factor (unpivoted, blocked)
//   rank t1 from R_y's column tails    hqr_factor (posterior range estimate)
//   Q1 = Q_y [I_t1; 0]                 hqr_apply
//   B^T = C^T Q1 = Q_b R_b             hqr_factor
//   R_b Pi = Q_r R_r, truncated at k   qrcp_reg (pivoting on a t1 x t1 matrix)
//   V~ = Q_b [Q_r; 0],  U = Q1 Pi R_r[:k,:]^T
//
// Column pivoting is invariant under the orthogonal factor, so pivoting R_b
// selects what pivoting B^T would.
//
// hqr_factor: one 512-thread workgroup per matrix (m <= 1024 rows).  Panels of
// 16 columns are factored in registers (two barriers per column); the
// compact-WY factor T (Schreiber-Van Loan: Q_p = I - V T V^T) is built from
// the Gram matrix V^T V; the trailing columns are updated 16 at a time as
// A -= V (T^T (V^T A)), both products on v_mfma_f64_16x16x4f64, the K = rows
// reduction of V^T A split over the 8 waves, the panel V resident in LDS.
//
// MFMA lane layout (measured on gfx950): D = X Y + C with X[i][k] in lane
// i + 16k, Y[k][j] in lane j + 16k, D[i][j] in lane j + 16 (i mod 4),
// register i / 4.
#include "kernels.h"
#include "compress.h"
#include "wave.h"

namespace tlrk {

typedef double d4 __attribute__((ext_vector_type(4)));

// Global-memory views of the task pointers.  The tasks live in device memory,
// so a plain pointer read from one could name any address space as far as
// the compiler knows, and it emits flat loads and stores.  Flat operations
// also count against the LDS counter: each wait for an LDS read would then
// wait for the outstanding global traffic too.  Every task pointer addresses
// global memory (device or host-mapped; never LDS or scratch).
typedef __attribute__((address_space(1))) double gdouble;
template <class T>
__device__ inline __attribute__((address_space(1))) T* gptr(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

namespace {

constexpr int NT = 512;                 // threads per workgroup
constexpr int NW = NT / 64;             // wave64s
constexpr int PB = 16;                  // panel width
constexpr int LDP = kQrMaxRows + 2;     // LDS panel stride (2 mod 32 doubles: conflict-free fragments)
constexpr int MB = kQrMaxRows / (NW * 16);   // 16-row blocks per wave
constexpr int RS = 16 * 17;             // per-wave slot of `red`: a 16 x 17 tile or a 16 x 16 partial

__device__ inline d4 mfma(double x, double y, d4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, c, 0, 0, 0); }

// Householder vector entry V[r][c] of panel c0 (unit lower trapezoidal).
__device__ inline double vval_lds(const double* P, int r, int c, int mm, bool live) {
  if (!live || r >= mm || r < c) return 0.0;
  return r == c ? 1.0 : P[c * LDP + r];
}


// One trailing-update round on the 16 columns col0.. of M (rows c0.., mm of
// them; ncol columns in all): M -= V op(T) (V^T M), op(T) = T^T (applying
// Q^T) or T (applying Q).  vx: this wave's V fragments in the X-layout of
// V^T M (registers); the Y-layout fragments of V W' are read from the panel P
// in LDS.  Each wave reads its rows of the chunk once, coalesced, into
// registers (the D-layout of the update product) and transposes them block by
// block through a wave-private 16 x 17 LDS tile (its slot of `red`) for
// V^T M.  Three barriers.
template <bool TRANS>
__device__ inline void wy_update(gdouble* M, int64_t ldm, int c0, int mm, int col0, int ncol, int rb, int nblk,
                                 const double (&vx)[MB][4], const double* P, int nlive, double* red, double* Wf,
                                 double* Wp, const double* Ts, int tid, int lane, int w) {
  double* tile = red + w * RS;   // 16 x 17 transpose tile; later this wave's partial W
  d4 cd[MB];
  d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int b = 0; b < MB; ++b) {
    const int row = rb + 16 * b + (lane & 15);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int col = col0 + 4 * r + (lane >> 4);
      cd[b][r] = (b < nblk && row < mm && col < ncol) ? M[(int64_t)col * ldm + c0 + row] : 0.0;
    }
  }
#pragma unroll
  for (int b = 0; b < MB; ++b) {
    if (b < nblk) {
      // D-layout (row lane & 15, column 4r + (lane >> 4)) -> tile[col * 17 + row]
#pragma unroll
      for (int r = 0; r < 4; ++r) tile[(4 * r + (lane >> 4)) * 17 + (lane & 15)] = cd[b][r];
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int q = 0; q < 4; ++q) acc = mfma(vx[b][q], tile[(lane & 15) * 17 + 4 * q + (lane >> 4)], acc);
      __builtin_amdgcn_wave_barrier();
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) tile[(4 * r + (lane >> 4)) * 16 + (lane & 15)] = acc[r];
  __syncthreads();
  if (tid < 256) {
    double sacc = 0.0;
#pragma unroll
    for (int v = 0; v < NW; ++v) sacc += red[v * RS + tid];
    Wf[tid] = sacc;   // W[i][j], i = panel column, j = column col0 + j
  }
  __syncthreads();
  if (tid < 256) {
    const int k = tid >> 4, j = tid & 15;
    double sacc = 0.0;
    if (TRANS) {
#pragma unroll
      for (int l = 0; l < 16; ++l)
        if (l <= k) sacc += Ts[l * 16 + k] * Wf[l * 16 + j];
    } else {
#pragma unroll
      for (int l = 0; l < 16; ++l)
        if (l >= k) sacc += Ts[k * 16 + l] * Wf[l * 16 + j];
    }
    Wp[tid] = sacc;
  }
  __syncthreads();
  double xw[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) xw[q] = -Wp[(4 * q + (lane >> 4)) * 16 + (lane & 15)];
#pragma unroll
  for (int b = 0; b < MB; ++b) {
    if (b < nblk) {
      const int row = rb + 16 * b + (lane & 15);
      d4 c = cd[b];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int cy = 4 * q + (lane >> 4);
        c = mfma(xw[q], vval_lds(P, row, cy, mm, cy < nlive), c);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int col = col0 + 4 * r + (lane >> 4);
        if (row < mm && col < ncol) M[(int64_t)col * ldm + c0 + row] = c[r];
      }
    }
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// A = Q R in place: R in the upper triangle, the Householder vectors (unit
// diagonal implied) below it, T factors per panel in tk.T.  With tk.tol > 0
// also the range rank t1 = max_i t_i, t_i the first row from which column i's
// tail norm ||R[t:, i]|| stays <= tol: for t >= t1 every sample y_i with
// i >= t is reproduced by Q_y[:, :t] to within tol (a posteriori estimate of
// ||(I - Q Q^T) C||, Halko-Martinsson-Tropp).  flag = 1 when fewer than
// min_tail samples back that estimate (and t1 < m).
//
// The panel is factored in registers (thread: rows tid, tid + 512); per
// column one batched reduction (the norm and the 15 reflector products
// together), finished across waves through 8 LDS partials.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(NT) hqr_factor_kernel(const HqrTask* __restrict__ tasks) {
  const HqrTask tk = tasks[blockIdx.x];
  __shared__ double P[PB * LDP];   // the panel
  __shared__ double red[NW * RS];
  __shared__ double Wf[256], Wp[256], Ts[256];
  __shared__ double taus[PB];
  __shared__ double dred[2 * NW * PB];   // per-wave column sums, two buffers (by column parity)
  __shared__ double rowc[2 * PB];        // row c of the panel, two buffers
  __shared__ int sh_t1;

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int m = tk.m, s = tk.s;
  if (m <= 0 || s <= 0) {
    if (tid == 0) {
      if (tk.rank) *tk.rank = 0;
      if (tk.flag) *tk.flag = 0;
    }
    return;
  }
  gdouble* A = gptr(tk.A);
  const int64_t lda = tk.lda;
  const int nref = m < s ? m : s;
  const int np = (nref + PB - 1) / PB;
  const int r0 = tid, r1 = tid + NT;

  for (int p = 0; p < np; ++p) {
    const int c0 = p * PB;
    const int mm = m - c0;
    const int pw = (s - c0) < PB ? (s - c0) : PB;
    // 1. panel -> registers
    double a0[PB], a1[PB];
#pragma unroll
    for (int c = 0; c < PB; ++c) {
      const gdouble* ac = A + (int64_t)(c0 + c) * lda + c0;
      a0[c] = (c < pw && r0 < mm) ? ac[r0] : 0.0;
      a1[c] = (c < pw && r1 < mm) ? ac[r1] : 0.0;
    }
    // 2. factor the panel.  Column c's reflector and its products with the
    // columns k > c come from one reduction: with x = A[c:, c], alpha = x_c,
    // sigma = |x_{>c}|^2 and p_k = x_{>c}^T A[>c, k], the reflector
    // v = (x - beta e_c) / (alpha - beta) has v^T A[c:, k] = A[c, k] +
    // p_k / (alpha - beta).  So each column costs one barrier.
#pragma unroll
    for (int c = 0; c < PB; ++c) {
      if (c0 + c < nref) {
        const double x0 = a0[c], x1 = a1[c];
        const double y0 = (r0 > c) ? x0 : 0.0;   // rows below c
        double part[16];
#pragma unroll
        for (int k = 0; k < 16; ++k)
          part[k] = (k == c) ? y0 * x0 + x1 * x1 : (k > c ? y0 * a0[k] + x1 * a1[k] : 0.0);
        const double tot = wave::bfly<16>(part, lane);
        double* dr = dred + (c & 1) * NW * PB;
        double* rc = rowc + (c & 1) * PB;
        if ((lane & 3) == 0) dr[w * PB + ((lane >> 2) & 15)] = tot;
        if (tid == c) {
#pragma unroll
          for (int k = 0; k < 16; ++k) rc[k] = a0[k];
        }
        __syncthreads();
        const int kl = lane & 15;
        double sk = 0.0;   // lane kl: sigma (kl == c) or p_kl
#pragma unroll
        for (int v = 0; v < NW; ++v) sk += dr[v * PB + kl];
        const double sig = wave::read(sk, c);
        const double alpha = rc[c];
        double ta, beta, sc;
        if (sig == 0.0) {
          ta = 0.0; beta = alpha; sc = 0.0;
        } else {
          const double nx = sqrt(alpha * alpha + sig);
          beta = alpha >= 0.0 ? -nx : nx;
          ta = (beta - alpha) / beta;
          sc = 1.0 / (alpha - beta);
        }
        const double dl = ta * (rc[kl] + sc * sk);   // lane k: tau v^T A[c:, k]
        const double v0 = (r0 > c) ? x0 * sc : (r0 == c ? 1.0 : 0.0);
        const double v1 = x1 * sc;
        a0[c] = (r0 == c) ? beta : (r0 > c ? v0 : x0);
        a1[c] = v1;
        if (tid == 0) taus[c] = ta;
#pragma unroll
        for (int k = 0; k < 16; ++k)
          if (k > c) {
            const double dk = wave::read(dl, k);
            a0[k] -= dk * v0;
            a1[k] -= dk * v1;
          }
      } else if (tid == 0) {
        taus[c] = 0.0;
      }
    }
    // 3. panel -> LDS and A (R above and on the diagonal, reflectors below)
#pragma unroll
    for (int c = 0; c < PB; ++c) {
      if (r0 < mm) P[c * LDP + r0] = a0[c];
      if (r1 < mm) P[c * LDP + r1] = a1[c];
      gdouble* ac = A + (int64_t)(c0 + c) * lda + c0;
      if (c < pw && r0 < mm) ac[r0] = a0[c];
      if (c < pw && r1 < mm) ac[r1] = a1[c];
    }
    __syncthreads();
    // 4. V fragments and the Gram matrix G = V^T V
    const int rw = ((mm + NW * 16 - 1) / (NW * 16)) * 16;
    const int nblk = rw / 16;
    const int rb = w * rw;
    const int nlive = nref - c0;
    double vx[MB][4];
    d4 g = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int b = 0; b < MB; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int cx = lane & 15;
        vx[b][q] = (b < nblk) ? vval_lds(P, rb + 16 * b + 4 * q + (lane >> 4), cx, mm, cx < nlive) : 0.0;
        if (b < nblk) g = mfma(vx[b][q], vx[b][q], g);
      }
#pragma unroll
    for (int r = 0; r < 4; ++r) red[w * RS + (4 * r + (lane >> 4)) * 16 + (lane & 15)] = g[r];
    __syncthreads();
    if (tid < 256) {
      double sacc = 0.0;
#pragma unroll
      for (int v = 0; v < NW; ++v) sacc += red[v * RS + tid];
      Wf[tid] = sacc;
    }
    __syncthreads();
    // T (upper triangular): T[i][i] = tau_i, T[0:i, i] = -tau_i T[0:i, 0:i] G[0:i, i]
    if (w == 0 && lane < 16) {
      double tr[16] = {};
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        double acc = 0.0;
#pragma unroll
        for (int l = 0; l < 16; ++l)
          if (l < i && l >= lane) acc += tr[l] * Wf[l * 16 + i];
        const double ti = taus[i];
        tr[i] = (lane < i) ? -ti * acc : (lane == i ? ti : 0.0);
      }
#pragma unroll
      for (int l = 0; l < 16; ++l) {
        Ts[lane * 16 + l] = tr[l];
        gptr(tk.T)[(int64_t)p * 256 + lane * 16 + l] = tr[l];
      }
    }
    __syncthreads();
    // 5. trailing columns: A -= V T^T V^T A
    for (int col0 = c0 + PB; col0 < s; col0 += PB)
      wy_update<true>(A, lda, c0, mm, col0, s, rb, nblk, vx, P, nlive, red, Wf, Wp, Ts, tid, lane, w);
    __syncthreads();
  }

  if (tk.tol > 0.0 && tk.trunc) {
    // Truncation rank from the unpivoted R: dropping rows k.. of R leaves an
    // error of ||R[k:, k:]||_F = sqrt(sum_{r >= k} ||R[r, r:]||^2).  One pass
    // over the upper triangle (wave w: columns w, w + 8, ..; lane: rows
    // lane + 64 i) gives the per-row partial sums and writes Z; the panel
    // LDS, no longer needed, holds the partials of the 8 waves.
    constexpr int RI = kQrMaxCols / 64;
    constexpr int CB = 4;   // columns per batch of loads
    double part[RI];
#pragma unroll
    for (int i = 0; i < RI; ++i) part[i] = 0.0;
    const int zr = tk.Z ? (nref < tk.zcap ? nref : tk.zcap) : 0;
    gdouble* Z = gptr(tk.Z);
    for (int cb = w; cb < s; cb += NW * CB) {
      double v[CB][RI];
#pragma unroll
      for (int u = 0; u < CB; ++u) {
        const int c = cb + NW * u;
        const gdouble* ac = A + (int64_t)c * lda;
#pragma unroll
        for (int i = 0; i < RI; ++i) {
          const int r = lane + 64 * i;
          v[u][i] = (64 * i < nref && c < s && r <= c && r < nref) ? ac[r] : 0.0;
        }
      }
#pragma unroll
      for (int u = 0; u < CB; ++u) {
        const int c = cb + NW * u;
#pragma unroll
        for (int i = 0; i < RI; ++i) {
          const int r = lane + 64 * i;
          part[i] += v[u][i] * v[u][i];
          if (64 * i < zr && c < s && r < zr) Z[(int64_t)r * tk.ldz + c] = v[u][i];
        }
      }
    }
    double* rs = P;   // [NW][kQrMaxCols]
#pragma unroll
    for (int i = 0; i < RI; ++i) rs[w * kQrMaxCols + lane + 64 * i] = part[i];
    __syncthreads();
    if (w == 0) {
      // lane l scans rows 8l .. 8l + 7: suffix sums within the lane, then
      // over the lanes above it
      constexpr int RL = kQrMaxCols / 64;
      double f[RL];
#pragma unroll
      for (int j = 0; j < RL; ++j) {
        const int r = RL * lane + j;
        double acc = 0.0;
#pragma unroll
        for (int v2 = 0; v2 < NW; ++v2) acc += rs[v2 * kQrMaxCols + r];
        f[j] = r < nref ? acc : 0.0;
      }
#pragma unroll
      for (int j = RL - 2; j >= 0; --j) f[j] += f[j + 1];
      double suf = f[0];   // inclusive suffix over lanes >= lane
      for (int off = 1; off < 64; off <<= 1) {
        const double o = __shfl_down(suf, off, 64);
        if (lane + off < 64) suf += o;
      }
      const double above = suf - f[0];
      const double tol2 = tk.tol * tk.tol;
      int k = 0;
#pragma unroll
      for (int j = 0; j < RL; ++j)
        if (RL * lane + j < nref && f[j] + above > tol2) k = RL * lane + j + 1;
      for (int off = 32; off > 0; off >>= 1) {
        const int o = __shfl_xor(k, off, 64);
        k = o > k ? o : k;
      }
      if (lane == 0) {
        if (tk.rank) *tk.rank = k;
        if (tk.flag) *tk.flag = 0;
      }
    }
  } else if (tk.tol > 0.0) {
    if (tid == 0) sh_t1 = 0;
    __syncthreads();
    const double tol2 = tk.tol * tk.tol;
    for (int i = tid; i < s; i += NT) {
      const int top = i < m - 1 ? i : m - 1;
      const gdouble* ci = A + (int64_t)i * lda;
      double acc = 0.0;
      int ti = top + 1;
      for (int l = top; l >= 0; --l) {
        acc += ci[l] * ci[l];
        if (acc > tol2) break;
        ti = l;
      }
      atomicMax(&sh_t1, ti);
    }
    __syncthreads();
    if (tid == 0) {
      const int t1 = sh_t1;
      if (tk.rank) *tk.rank = t1;
      if (tk.flag) *tk.flag = (t1 < m && s - t1 < tk.min_tail) ? 1 : 0;
    }
  } else if (tid == 0) {
    if (tk.rank) *tk.rank = nref;
    if (tk.flag) *tk.flag = 0;
  }
}

// ---------------------------------------------------------------------------
// X <- Q X with Q = H_1 ... H_np from hqr_factor (X: m x kx, ldx).  identity:
// X starts as [I_kx; 0] (then only columns >= c0 change in panel c0);
// otherwise rows >= xrows of X are cleared first.
// ---------------------------------------------------------------------------
// Workgroup (task, y) applies Q to columns [y * kApplyCols, (y + 1) *
// kApplyCols) of X: the columns are independent, so a wide X (the largest
// tile of a column sets the launch time) is spread over several CUs.
__global__ void __launch_bounds__(NT) hqr_apply_kernel(const HqrTask* __restrict__ tasks,
                                                       const int* __restrict__ items) {
  // items (optional): workgroup b takes task items[2b], column chunk items[2b + 1]
  const int ti = items ? items[2 * blockIdx.x] : (int)blockIdx.x;
  const int cy = items ? items[2 * blockIdx.x + 1] : (int)blockIdx.y;
  const HqrTask tk = tasks[ti];
  __shared__ double P[PB * LDP];
  __shared__ double red[NW * RS];
  __shared__ double Wf[256], Wp[256], Ts[256];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int m = tk.m, s = tk.s;
  const int x0 = cy * kApplyCols;
  const int kx = tk.kx < x0 + kApplyCols ? tk.kx : x0 + kApplyCols;   // this workgroup: columns [x0, kx)
  if (m <= 0 || kx <= x0) return;
  gdouble* X = gptr(tk.X);
  const int64_t ldx = tk.ldx;
  const gdouble* A = gptr(tk.A);
  const int64_t lda = tk.lda;
  if (tk.identity) {
    for (int c = x0; c < kx; ++c)
      for (int r = tid; r < m; r += NT) X[(int64_t)c * ldx + r] = (r == c) ? 1.0 : 0.0;
  } else {
    const int rz = tk.xrows < 0 ? 0 : tk.xrows;
    for (int c = x0; c < kx; ++c)
      for (int r = rz + tid; r < m; r += NT) X[(int64_t)c * ldx + r] = 0.0;
  }
  const int nref = m < s ? m : s;
  const int np = (nref + PB - 1) / PB;
  for (int p = np - 1; p >= 0; --p) {
    const int c0 = p * PB;
    if (tk.identity && c0 >= kx) continue;   // columns left of the panel are still unit vectors
    const int mm = m - c0;
    const int nlive = nref - c0;
    __syncthreads();   // previous panel done with P, Ts and X
    if (tid < 256) Ts[tid] = gptr(tk.T)[(int64_t)p * 256 + tid];
#pragma unroll
    for (int c = 0; c < PB; ++c) {
      const gdouble* ac = A + (int64_t)(c0 + c) * lda + c0;
      for (int r = tid; r < mm; r += NT) P[c * LDP + r] = (c < nlive) ? ac[r] : 0.0;
    }
    __syncthreads();
    const int rw = ((mm + NW * 16 - 1) / (NW * 16)) * 16;
    const int nblk = rw / 16;
    const int rb = w * rw;
    double vx[MB][4];
#pragma unroll
    for (int b = 0; b < MB; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int cx = lane & 15;
        vx[b][q] = (b < nblk) ? vval_lds(P, rb + 16 * b + 4 * q + (lane >> 4), cx, mm, cx < nlive) : 0.0;
      }
    for (int col0 = (tk.identity && c0 > x0) ? c0 : x0; col0 < kx; col0 += PB)
      wy_update<false>(X, ldx, c0, mm, col0, kx, rb, nblk, vx, P, nlive, red, Wf, Wp, Ts, tid, lane, w);
  }
}

// ---------------------------------------------------------------------------
// Column-pivoted Householder QR of a small matrix (m, q <= kRegQrBig) held
// on chip: wave w owns columns w + 8j, lane l rows l + 64i.  Same stopping
// rule and outputs as qrcp_kernel (rank, Z, explicit Q), reading Y (only its
// upper triangle when tk.upper) and writing reflectors to the workspace W.
// Each step: the pivot column's wave forms the reflector (one barrier), every
// wave reflects its live columns and recomputes their norms with two batched
// wave reductions (one barrier).
//
// Up to kRegQrMax rows and columns the matrix is all in registers.  Beyond
// that (the range ranks of the tangent tiles next to the diagonal reach
// ~220) the extra rows (one per lane l < kXr) and the extra column slots of
// each wave live in LDS; every such element is read and written only by the
// thread that owns it, so the LDS share acts as more registers and needs no
// barriers of its own.
// ---------------------------------------------------------------------------
namespace {
constexpr int RIR = kRegQrMax / 64;                  // row slots per lane in registers
constexpr int RJR = kRegQrMax / NW;                  // column slots per wave in registers
constexpr int kXr = kRegQrBig - kRegQrMax;           // extra rows, one per lane l < kXr
constexpr int kXc = (kRegQrBig - kRegQrMax) / NW;    // extra column slots per wave
static_assert(kRegQrMax % 64 == 0 && kRegQrMax % NW == 0, "register block must tile the wave layout");
static_assert(kXr > 0 && kXr <= 64 && kXc * NW == kXr, "extra rows and columns must fit one slot each");
static_assert(RJR + kXc <= 32, "column slots must fit two 16-entry butterflies");

// One lane's share of the matrix: element (row lane + 64 i, column w + NW j).
template <bool BIG>
struct QrShare {
  static constexpr int RJ = BIG ? RJR + kXc : RJR;
  static constexpr int RI = BIG ? RIR + 1 : RIR;
  double r[RJR][RIR];
  double* xr;   // LDS [kRegQrBig][kXr]: row kRegQrMax + l of column c at c * kXr + l
  double* xc;   // LDS [kXc][NW][kRegQrMax]: extra column slot s of wave w, row r
  int w, lane;
  __device__ __forceinline__ double get(int j, int i) const {
    if (j < RJR && i < RIR) return r[j][i];
    if (i >= RIR) return lane < kXr ? xr[(w + NW * j) * kXr + lane] : 0.0;
    return xc[((j - RJR) * NW + w) * kRegQrMax + lane + 64 * i];
  }
  __device__ __forceinline__ void set(int j, int i, double v) {
    if (j < RJR && i < RIR) {
      r[j][i] = v;
    } else if (i >= RIR) {
      if (lane < kXr) xr[(w + NW * j) * kXr + lane] = v;
    } else {
      xc[((j - RJR) * NW + w) * kRegQrMax + lane + 64 * i] = v;
    }
  }
};

struct QrShared {
  double* vs;       // reflector of the current step, 64 * (RIR + 1) rows
  double* taus;     // [kRegQrBig]
  int* step_of;     // [kRegQrBig]
  double* wsum;     // [NW] per-wave sum / max / argmax of the live column norms
  double* wmax;
  int* widx;
  double* xr;
  double* xc;
};

template <bool BIG>
__device__ __forceinline__ void qrcp_reg_body(const QrcpTask& tk, const QrShared& sh) {
  using Share = QrShare<BIG>;
  constexpr int RJ = Share::RJ, RI = Share::RI;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int m = tk.m, q = tk.q;
  double* vs = sh.vs;
  double* taus = sh.taus;
  int* step_of = sh.step_of;
  const gdouble* Y = gptr(tk.Y);
  const int64_t ldy = tk.ldy;
  Share a;
  a.xr = sh.xr;
  a.xc = sh.xc;
  a.w = w;
  a.lane = lane;
#pragma unroll
  for (int j = 0; j < RJ; ++j) {
    const int c = w + NW * j;
#pragma unroll
    for (int i = 0; i < RI; ++i) {
      const int r = lane + 64 * i;
      a.set(j, i, (c < q && r < m && (!tk.upper || r <= c)) ? Y[(int64_t)c * ldy + r] : 0.0);
    }
  }
  for (int c = tid; c < kRegQrBig; c += NT) step_of[c] = 0x7fffffff;
  uint32_t done = 0;   // bit j: column w + 8j already pivoted

  // Sums over the wave of per-column partials f(j), j < RJ, in two 16-entry
  // butterflies: lanes with (lane & 3) == 0 end with the totals of columns
  // slot e and 16 + e, e = (lane >> 2) & 15.
  auto reduce_cols = [&](auto f, double& lo, double& hi) {
    double part[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) part[j] = (j < RJ) ? f(j) : 0.0;
    lo = wave::bfly<16>(part, lane);
#pragma unroll
    for (int j = 0; j < 16; ++j) part[j] = (16 + j < RJ) ? f(16 + j) : 0.0;
    hi = wave::bfly<16>(part, lane);
  };
  // per-wave norm statistics of the live columns over rows > t (t = -1: all)
  auto norms = [&](int t) {
    double lo, hi;
    reduce_cols([&](int j) {
      double acc = 0.0;
#pragma unroll
      for (int i = 0; i < RI; ++i)
        if (lane + 64 * i > t) {
          const double v = a.get(j, i);
          acc += v * v;
        }
      return acc;
    }, lo, hi);
    const int e = (lane >> 2) & 15;
    double mv = -1.0, sv = 0.0;
    int mi = 0x7fffffff;
#pragma unroll
    for (int h2 = 0; h2 < 2; ++h2) {
      const int es = e + 16 * h2;
      const int ce = w + NW * es;
      const double v = h2 ? hi : lo;
      if ((lane & 3) == 0 && es < RJ && ce < q && !((done >> es) & 1u)) {
        sv += v;
        if (v > mv || (v == mv && ce < mi)) { mv = v; mi = ce; }
      }
    }
    wave::max_sum(mv, mi, sv, lane);
    if (lane == 0) { sh.wsum[w] = sv; sh.wmax[w] = mv; sh.widx[w] = mi; }
  };
  norms(-1);
  __syncthreads();

  const int tmax = m < q ? m : q;
  const double tol2 = tk.tol * tk.tol;
  int t = 0;
  for (; t < tmax; ++t) {
    double total = 0.0, best = -1.0;
    int p = 0x7fffffff;
#pragma unroll
    for (int v = 0; v < NW; ++v) {
      total += sh.wsum[v];
      if (sh.wmax[v] > best || (sh.wmax[v] == best && sh.widx[v] < p)) { best = sh.wmax[v]; p = sh.widx[v]; }
    }
    if (total <= tol2 || t >= tk.max_rank || p >= q) break;
    const int pw = p % NW, pj = p / NW;
    if (w == pw) {
      double x[RI];
#pragma unroll
      for (int i = 0; i < RI; ++i) {
        x[i] = 0.0;
#pragma unroll
        for (int j = 0; j < RJ; ++j)
          if (j == pj) x[i] = a.get(j, i);
      }
      double sq = 0.0;
#pragma unroll
      for (int i = 0; i < RI; ++i)
        if (lane + 64 * i > t) sq += x[i] * x[i];
      sq = wave::sum(sq);
      double xs = x[0];
#pragma unroll
      for (int i = 1; i < RI; ++i)
        if ((t >> 6) == i) xs = x[i];
      const double alpha = wave::read(xs, t & 63);
      double ta, beta, sc;
      if (sq == 0.0) {
        ta = 0.0; beta = alpha; sc = 0.0;
      } else {
        const double nx = sqrt(alpha * alpha + sq);
        beta = alpha >= 0.0 ? -nx : nx;
        ta = (beta - alpha) / beta;
        sc = 1.0 / (alpha - beta);
      }
#pragma unroll
      for (int i = 0; i < RI; ++i) {
        const int r = lane + 64 * i;
        const double v = (r > t) ? x[i] * sc : (r == t ? 1.0 : 0.0);
        vs[r] = v;
        const double nv = (r == t) ? beta : (r > t ? v : x[i]);
#pragma unroll
        for (int j = 0; j < RJ; ++j)
          if (j == pj) a.set(j, i, nv);
      }
      if (lane == 0) { taus[t] = ta; step_of[p] = t; }
    }
    done |= (pw == w) ? (1u << pj) : 0u;
    __syncthreads();
    const double ta = taus[t];
    double vv[RI];
#pragma unroll
    for (int i = 0; i < RI; ++i) vv[i] = vs[lane + 64 * i];
    double lo, hi;
    reduce_cols([&](int j) {
      double acc = 0.0;
      if (!((done >> j) & 1u)) {
#pragma unroll
        for (int i = 0; i < RI; ++i) acc += vv[i] * a.get(j, i);
      }
      return acc;
    }, lo, hi);
#pragma unroll
    for (int j = 0; j < RJ; ++j) {
      const double d = ta * wave::read(j < 16 ? lo : hi, 4 * (j & 15));
      if (!((done >> j) & 1u)) {
#pragma unroll
        for (int i = 0; i < RI; ++i) a.set(j, i, a.get(j, i) - d * vv[i]);
      }
    }
    norms(t);
    __syncthreads();
  }
  const int rank = t;
  if (tid == 0) {
    if (tk.rank) *tk.rank = rank;
    if (tk.flag) *tk.flag = (q - rank < tk.min_tail) ? 1 : 0;
  }
  // Z[c, rr] = R[rr, step_of[c]]; reflector of step st -> W column st
#pragma unroll
  for (int j = 0; j < RJ; ++j) {
    const int c = w + NW * j;
    if (c >= q) continue;
    const int st = step_of[c];
#pragma unroll
    for (int i = 0; i < RI; ++i) {
      const int r = lane + 64 * i;
      if (r >= m) continue;
      const double v = a.get(j, i);
      if (tk.Z && r < rank) gptr(tk.Z)[(int64_t)r * tk.ldz + c] = (st >= r) ? v : 0.0;
      if (st < rank) gptr(tk.W)[(int64_t)st * tk.ldw + r] = (r > st) ? v : 0.0;
    }
  }
  if (tk.tau)
    for (int i = tid; i < rank; i += NT) gptr(tk.tau)[i] = taus[i];
  if (!tk.Q || rank == 0) return;
  __syncthreads();
  // explicit Q = H_0 ... H_{rank-1} [I; 0]: column c still equals e_c before
  // step st <= c is applied, so step st only touches columns >= st.  The
  // share is reused (each thread rewrites only its own elements).
  Share qa;
  qa.xr = sh.xr;
  qa.xc = sh.xc;
  qa.w = w;
  qa.lane = lane;
#pragma unroll
  for (int j = 0; j < RJ; ++j)
#pragma unroll
    for (int i = 0; i < RI; ++i) qa.set(j, i, (lane + 64 * i == w + NW * j) ? 1.0 : 0.0);
  for (int st = rank - 1; st >= 0; --st) {
    const double ta = taus[st];
    double vv[RI];
#pragma unroll
    for (int i = 0; i < RI; ++i) {
      const int r = lane + 64 * i;
      vv[i] = (r == st) ? 1.0 : ((r > st && r < m) ? gptr(tk.W)[(int64_t)st * tk.ldw + r] : 0.0);
    }
    double lo, hi;
    reduce_cols([&](int j) {
      double acc = 0.0;
      const int c = w + NW * j;
      if (c >= st && c < rank) {
#pragma unroll
        for (int i = 0; i < RI; ++i) acc += vv[i] * qa.get(j, i);
      }
      return acc;
    }, lo, hi);
#pragma unroll
    for (int j = 0; j < RJ; ++j) {
      const int c = w + NW * j;
      const double d = ta * wave::read(j < 16 ? lo : hi, 4 * (j & 15));
      if (c >= st && c < rank) {
#pragma unroll
        for (int i = 0; i < RI; ++i) qa.set(j, i, qa.get(j, i) - d * vv[i]);
      }
    }
  }
#pragma unroll
  for (int j = 0; j < RJ; ++j) {
    const int c = w + NW * j;
    if (c >= rank) continue;
#pragma unroll
    for (int i = 0; i < RI; ++i) {
      const int r = lane + 64 * i;
      if (r < m) gptr(tk.Q)[(int64_t)c * tk.ldq + r] = qa.get(j, i);
    }
  }
}
}  // namespace

__global__ void __launch_bounds__(NT) qrcp_reg_kernel(const QrcpTask* __restrict__ tasks) {
  const QrcpTask tk = tasks[blockIdx.x];
  __shared__ double vs[64 * (RIR + 1)];
  __shared__ double taus[kRegQrBig];
  __shared__ int step_of[kRegQrBig];
  __shared__ double wsum[NW], wmax[NW];
  __shared__ int widx[NW];
  __shared__ double xr[kRegQrBig * kXr];
  __shared__ double xc[kXc * NW * kRegQrMax];
  const int m = tk.m, q = tk.q;
  if (m <= 0 || q <= 0 || m > kRegQrBig || q > kRegQrBig) {   // the host routes larger ones to qrcp_kernel
    if (threadIdx.x == 0) {
      if (tk.rank) *tk.rank = 0;
      if (tk.flag) *tk.flag = (m > 0 && q > 0) ? 1 : 0;
    }
    return;
  }
  const QrShared sh{vs, taus, step_of, wsum, wmax, widx, xr, xc};
  if (m <= kRegQrMax && q <= kRegQrMax) qrcp_reg_body<false>(tk, sh);
  else qrcp_reg_body<true>(tk, sh);
}

// Upper-triangular copy (zeros below the diagonal) of rows/cols [0, n_b) of
// batched square blocks; grid.y = batch.
__global__ void copy_upper_kernel(const double* __restrict__ src, int64_t sld, const int64_t* __restrict__ soff,
                                  double* __restrict__ dst, int64_t dld, const int64_t* __restrict__ doff,
                                  const int* __restrict__ nn) {
  const int b = blockIdx.y;
  const int n = nn[b];
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)n * n) return;
  const int64_t r = e % n, c = e / n;
  dst[doff[b] + c * dld + r] = (r <= c) ? src[soff[b] + c * sld + r] : 0.0;
}

// ---------------------------------------------------------------------------
// Compact-WY factor of reflectors 16p .. 16p + 15 (workgroup (task, p)): the
// Gram matrix G = V^T V of the unit lower trapezoidal V, staged through LDS
// 256 rows at a time, then T[i][i] = tau_i, T[0:i, i] = -tau_i T[0:i, 0:i]
// G[0:i, i] (Schreiber-Van Loan), as hqr_factor builds it.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) wy_build_kernel(const HqrTask* __restrict__ tasks) {
  const HqrTask tk = tasks[blockIdx.x];
  const int p = blockIdx.y;
  const int nref = tk.m < tk.s ? tk.m : tk.s;
  const int c0 = PB * p;
  if (c0 >= nref) return;   // uniform over the workgroup
  const int nlive = nref - c0 < PB ? nref - c0 : PB;
  const int mm = tk.m - c0;
  __shared__ double V[PB][257];
  __shared__ double G[PB * PB];
  const int tid = threadIdx.x;
  const int a = tid >> 4, b = tid & 15;
  double g = 0.0;
  for (int r0 = 0; r0 < mm; r0 += 256) {
    const int r = r0 + tid;
#pragma unroll
    for (int c = 0; c < PB; ++c) {
      double v = 0.0;
      if (c < nlive && r < mm) v = (r == c) ? 1.0 : (r > c ? gptr(tk.A)[(int64_t)(c0 + c) * tk.lda + c0 + r] : 0.0);
      V[c][tid] = v;
    }
    __syncthreads();
    const int rn = mm - r0 < 256 ? mm - r0 : 256;
    for (int q = 0; q < rn; ++q) g += V[a][q] * V[b][q];
    __syncthreads();
  }
  G[a * PB + b] = g;
  __syncthreads();
  if (tid < PB) {
    const int lane = tid;
    double tr[PB] = {};
#pragma unroll
    for (int i = 0; i < PB; ++i) {
      double acc = 0.0;
#pragma unroll
      for (int l = 0; l < PB; ++l)
        if (l < i && l >= lane) acc += tr[l] * G[l * PB + i];
      const double ti = (i < nlive) ? gptr(tk.tau)[c0 + i] : 0.0;
      tr[i] = (lane < i) ? -ti * acc : (lane == i ? ti : 0.0);
    }
#pragma unroll
    for (int l = 0; l < PB; ++l) gptr(tk.T)[(int64_t)p * 256 + lane * PB + l] = tr[l];
  }
}

hipError_t launch_wy_build(const HqrTask* d_tasks, int count, hipStream_t s, int max_s) {
  if (count <= 0 || max_s <= 0) return hipSuccess;
  hipLaunchKernelGGL(wy_build_kernel, dim3((unsigned)count, (unsigned)((max_s + PB - 1) / PB)), dim3(256), 0, s,
                     d_tasks);
  return hipGetLastError();
}

hipError_t launch_hqr_factor(const HqrTask* d_tasks, int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(hqr_factor_kernel, dim3((unsigned)count), dim3(NT), 0, s, d_tasks);
  return hipGetLastError();
}

hipError_t launch_hqr_apply(const HqrTask* d_tasks, int count, hipStream_t s, int max_kx, const int* d_items,
                            int nitems) {
  if (d_items) {
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(hqr_apply_kernel, dim3((unsigned)nitems), dim3(NT), 0, s, d_tasks, d_items);
    return hipGetLastError();
  }
  if (count <= 0) return hipSuccess;
  const int chunks = max_kx > kApplyCols ? (max_kx + kApplyCols - 1) / kApplyCols : 1;
  hipLaunchKernelGGL(hqr_apply_kernel, dim3((unsigned)count, (unsigned)chunks), dim3(NT), 0, s, d_tasks,
                     (const int*)nullptr);
  return hipGetLastError();
}

hipError_t launch_qrcp_reg(const QrcpTask* d_tasks, int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(qrcp_reg_kernel, dim3((unsigned)count), dim3(NT), 0, s, d_tasks);
  return hipGetLastError();
}

hipError_t launch_copy_upper(const double* src, int64_t sld, const int64_t* soff, double* dst, int64_t dld,
                             const int64_t* doff, const int* nn, int nmax, int count, hipStream_t s) {
  if (count <= 0 || nmax <= 0) return hipSuccess;
  const int64_t tot = (int64_t)nmax * nmax;
  hipLaunchKernelGGL(copy_upper_kernel, dim3((unsigned)((tot + 255) / 256), (unsigned)count), dim3(256), 0, s, src,
                     sld, soff, dst, dld, doff, nn);
  return hipGetLastError();
}

}  // namespace tlrk
