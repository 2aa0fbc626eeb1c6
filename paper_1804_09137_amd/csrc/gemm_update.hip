// Column-update GEMM for gfx950 (the left-looking update of Section V's TLR
// Cholesky, done by dense accumulation: C -= W U_row^T over the rows below the
// diagonal tile).
//
// MFMA lane layout of v_mfma_f64_16x16x4f64 (measured on gfx950): with the
// operands passed as (B fragment, A fragment), lane l of the result holds row
// (l & 15) and column (l >> 4) + 4 r of the 16 x 16 block in register r.
#include "kernels.h"

namespace tlrk {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kXcds = 8;   // workgroup w runs on XCD w mod 8

// ---------------------------------------------------------------------------
// Column-update GEMM: C = alpha A B^T + beta C with A (M x K) and B (N x K)
// column-major, FP64, N = 256 q or 256 q + 32 (the tile width).  A workgroup
// takes 128 rows by 256 columns (8 waves of 64 x 64); the workgroups of the
// last tile column also take the 32 columns beyond 256 q (each wave 16 rows
// of them), so all of N is one launch and the q workgroups of a row panel,
// consecutive on one XCD, stream that panel of A while it sits in L2.  K is
// consumed in 16-wide slices through three LDS stages filled by direct
// global-to-LDS loads (16 bytes a lane), issued two slices ahead of the
// MFMAs, so the operand loads need no registers and their latency hides
// behind two slices of MFMAs.  A workgroup whose rows run past M, and the
// partial last slice, load through registers with bounds masks instead.
// ---------------------------------------------------------------------------
namespace {
constexpr int UB_M = 128;    // rows per workgroup
constexpr int UB_N = 256;    // columns per workgroup (main block)
constexpr int UB_E = 32;     // extra columns of the last tile column
constexpr int UB_K = 16;     // K slice
constexpr int UB_NT = 512;   // 8 wave64s: 2 (rows) x 4 (columns) of 64 x 64
constexpr int UB_LOADS = 7;  // direct loads per wave and slice (2 A, 4 B, 1 extra)

struct UpdArgs {
  const double* A;  // M x K, ld lda
  const double* B;  // N x K, ld ldb
  double* C;        // M x N, ld ldc
  int64_t lda, ldb, ldc;
  int64_t M, N, K;
  int nq;           // 256-column tile columns
  int extra;        // 0 or 32: columns 256 nq .. N, taken by tile column nq - 1
  double alpha, beta;
  int64_t gx;       // row tiles
};

typedef __attribute__((address_space(3))) void lds_void;

// One direct global-to-LDS load, 16 bytes a lane: lane l's bytes land at
// lds_dst + 16 l (lds_dst uniform over the wave).  Inline asm, so that the
// compiler does not track it: its own tracking cannot tell the three stages
// apart and would wait for every load in flight before each LDS read.  The
// instruction has no register result; the kernel waits for it (vmcnt) and
// publishes the stage with the workgroup barrier.
__device__ __forceinline__ void upd_dma16(const double* src, double* lds_dst) {
  const uint32_t lds = (uint32_t)(uintptr_t)(lds_void*)lds_dst;
  asm volatile("s_mov_b32 m0, %1\n\tglobal_load_lds_dwordx4 %0, off" : : "v"(src), "s"(lds) : "memory", "m0");
}

// The workgroup barrier without a memory fence (a fence would wait for the
// direct loads in flight), fenced for the compiler only: no LDS access moves
// across it.
__device__ __forceinline__ void upd_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}
}  // namespace

__global__ void __launch_bounds__(UB_NT) gemm_update_kernel(UpdArgs g) {
  // one array per stage (A, then B, then the extra columns)
  constexpr int SB = UB_K * UB_M, SE = SB + UB_K * UB_N, SZ = SE + UB_K * UB_E;
  __shared__ double st0[SZ], st1[SZ], st2[SZ];

  // the wave index in a scalar register (the load addresses are a scalar
  // column start plus a per-lane offset)
  const int tid = threadIdx.x, lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = w & 1, wn = w >> 1;
  const int64_t total = g.gx * g.nq;
  const int64_t per = (total + kXcds - 1) / kXcds;
  const int64_t logical = (int64_t)(blockIdx.x % kXcds) * per + blockIdx.x / kXcds;
  if (logical >= total) return;
  const int64_t tm = logical / g.nq;
  const int tn = (int)(logical - tm * g.nq);
  const int64_t m0 = tm * UB_M, n0 = (int64_t)tn * UB_N;
  const bool has_e = g.extra > 0 && tn == g.nq - 1;
  const int64_t ne0 = (int64_t)g.nq * UB_N;   // first extra column
  const int64_t M = g.M, K = g.K;
  const double* __restrict__ A = g.A;
  const double* __restrict__ B = g.B;

  d4 acc[4][4];
  d4 acce[2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = d4{0, 0, 0, 0};
  acce[0] = acce[1] = d4{0, 0, 0, 0};

  // one slice from a stage; the fragments of the next k4 step are read while
  // the current one's MFMAs run
  auto compute = [&](const double* sa, const double* sb, const double* se) {
    double a[2][4], b[2][4];
    auto frag = [&](int k4, double (&aa)[4], double (&bb)[4]) {
      const int kr = k4 * 4 + (lane >> 4);
#pragma unroll
      for (int i = 0; i < 4; ++i) aa[i] = sa[kr * UB_M + wm * 64 + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 4; ++j) bb[j] = sb[kr * UB_N + wn * 64 + j * 16 + (lane & 15)];
    };
    frag(0, a[0], b[0]);
#pragma unroll
    for (int k4 = 0; k4 < UB_K / 4; ++k4) {
      const int c = k4 & 1;
      if (k4 + 1 < UB_K / 4) frag(k4 + 1, a[c ^ 1], b[c ^ 1]);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(b[c][j], a[c][i], acc[i][j], 0, 0, 0);
      if (has_e) {
        const int kr = k4 * 4 + (lane >> 4);
        const double ae = sa[kr * UB_M + w * 16 + (lane & 15)];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const double be = se[kr * UB_E + j * 16 + (lane & 15)];
          acce[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(be, ae, acce[j], 0, 0, 0);
        }
      }
    }
  };
  // bounds-masked register loads of the slice from column kc into one stage
  auto load_masked = [&](int64_t kc, double* sa, double* sb, double* se) {
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const int r = tid & 127, k = (tid >> 7) + 4 * p;
      sa[k * UB_M + r] = (m0 + r < M && kc + k < K) ? A[(m0 + r) + (kc + k) * g.lda] : 0.0;
    }
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      const int r = tid & 255, k = (tid >> 8) + 2 * p;
      sb[k * UB_N + r] = (kc + k < K) ? B[(n0 + r) + (kc + k) * g.ldb] : 0.0;
    }
    const int c = tid & 31, k = tid >> 5;
    se[k * UB_E + c] = (has_e && kc + k < K) ? B[(ne0 + c) + (kc + k) * g.ldb] : 0.0;
  };

  const bool direct = m0 + UB_M <= M;
  const int64_t nfull = direct ? K / UB_K : 0;
  // direct loads of full slice t into one stage: wave w takes A columns 2w
  // and 2w + 1, the same B columns (both halves) and four extra columns
  // (waves w and w + 4 load the same ones; a workgroup without extra columns
  // loads main columns there, so that every wave issues the same loads)
  auto issue = [&](int64_t t, double* sa, double* sb, double* se) {
    const int64_t kc = t * UB_K;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int k = 2 * w + i;
      const double* ca = A + m0 + (kc + k) * g.lda;
      const double* cb = B + n0 + (kc + k) * g.ldb;
      upd_dma16(ca + 2 * lane, sa + k * UB_M);
#pragma unroll
      for (int h = 0; h < 2; ++h) upd_dma16(cb + 128 * h + 2 * lane, sb + k * UB_N + 128 * h);
    }
    const int e = w & 3;
    const double* ce = B + (has_e ? ne0 : n0) + (kc + 4 * e) * g.ldb;
    upd_dma16(ce + (lane >> 4) * g.ldb + 2 * (lane & 15), se + 4 * e * UB_E);
  };
  // Step t waits for its own slice (all but the 7 loads of slice t + 1
  // complete), passes the barrier (slice t visible; every wave done with
  // slice t - 1, whose stage takes slice t + 2), issues slice t + 2 and
  // computes slice t.  Past the last slice the issue repeats the last slice
  // into the free stage, so that every step waits for the same count.  Steps
  // in groups of three: each stage is a fixed LDS array.
#define UPD_STEP(S, S2)                                                               \
  {                                                                                   \
    __builtin_amdgcn_s_waitcnt(0x0070 | UB_LOADS);                                    \
    upd_barrier();                                                                    \
    issue(t + 2 < nfull ? t + 2 : nfull - 1, st##S2, st##S2 + SB, st##S2 + SE);        \
    compute(st##S, st##S + SB, st##S + SE);                                           \
    ++t;                                                                              \
  }
  if (nfull >= 1) {
    issue(0, st0, st0 + SB, st0 + SE);
    issue(nfull > 1 ? 1 : 0, st1, st1 + SB, st1 + SE);
    for (int64_t t = 0; t < nfull;) {
      UPD_STEP(0, 2)
      if (t < nfull) UPD_STEP(1, 0)
      if (t < nfull) UPD_STEP(2, 1)
    }
    __builtin_amdgcn_s_waitcnt(0x0070);   // the repeated loads have landed too
  }
#undef UPD_STEP
  // the rest through registers: every slice of a workgroup past M, the
  // partial last slice otherwise
  for (int64_t t = nfull; t * UB_K < K; ++t) {
    const int s = (int)(t % 3);
    double* sa = s == 0 ? st0 : (s == 1 ? st1 : st2);
    __syncthreads();   // the stage's previous slice is consumed
    load_masked(t * UB_K, sa, sa + SB, sa + SE);
    __syncthreads();
    compute(sa, sa + SB, sa + SE);
  }

  // epilogue: lane holds rows .. + (lane & 15), columns .. + (lane >> 4) + 4 r
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t m = m0 + wm * 64 + i * 16 + (lane & 15);
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t n = n0 + wn * 64 + j * 16 + (lane >> 4) + 4 * r;
        if (m < M && n < g.N) {
          double* c = g.C + n * g.ldc + m;
          double o = g.alpha * acc[i][j][r];
          if (g.beta != 0.0) o += g.beta * (*c);
          *c = o;
        }
      }
  }
  if (has_e) {
    const int64_t m = m0 + w * 16 + (lane & 15);
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t n = ne0 + j * 16 + (lane >> 4) + 4 * r;
        if (m < M && n < g.N) {
          double* c = g.C + n * g.ldc + m;
          double o = g.alpha * acce[j][r];
          if (g.beta != 0.0) o += g.beta * (*c);
          *c = o;
        }
      }
  }
}

// gemm_update_kernel when the call fits it: one segment, both operands
// column-major with even leading dimensions and 16-byte aligned origins, N =
// 256 q or 256 q + 32, a linear epilogue (false: use the general kernels).
bool launch_gemm_update(const GemmSeg& sg, int64_t M, int64_t N, double* C, int64_t ldc, const GemmEpi& ep,
                               hipStream_t s, hipError_t* err) {
  const Operand& a = sg.A;
  const Operand& b = sg.B;
  const int64_t nq = N / UB_N, extra = N - nq * UB_N;
  if (ep.kind != kEpiLinear || a.layout != kContig || b.layout != kContig || sg.K <= 0 || M <= 0) return false;
  if (nq < 1 || (extra != 0 && extra != UB_E) || (a.ld & 1) || (b.ld & 1)) return false;
  const double* A = a.base + a.r0 + a.c0 * a.ld;
  const double* B = b.base + b.r0 + b.c0 * b.ld;
  if (((uintptr_t)A & 15) || ((uintptr_t)B & 15)) return false;
  UpdArgs g{A, B, C, a.ld, b.ld, ldc, M, N, sg.K, (int)nq, (int)extra, ep.alpha, ep.beta, (M + UB_M - 1) / UB_M};
  const int64_t total = g.gx * g.nq;
  const int64_t grid = ((total + kXcds - 1) / kXcds) * kXcds;
  if (grid > 0x7fffffff) return false;
  hipLaunchKernelGGL(gemm_update_kernel, dim3((unsigned)grid), dim3(UB_NT), 0, s, g);
  *err = hipGetLastError();
  return true;
}

}  // namespace tlrk
