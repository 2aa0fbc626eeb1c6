// FP64 MFMA GEMM for gfx950: C = epilogue(sum_s A_s B_s^T).
//
// A workgroup of WM x WN wave64s computes a BM x BN block of C with
// v_mfma_f64_16x16x4f64.  K is consumed in BK-wide slices staged through LDS
// (two stages for the large tiles, so one barrier per slice); the next slice
// is fetched into registers while the current one feeds the MFMAs.  The
// operand roles are swapped inside the MFMA (B feeds the 16-row side) so
// that each output register holds 16 consecutive rows of one column of the
// column-major C: stores are 128-byte runs.
//
// Generation epilogues (C = Matern - AB^T) are split off: a Matern kernel
// writes the block first and the GEMM then accumulates with alpha = -1,
// beta = 1.  Compiling the Matern evaluation into the MFMA kernel raised its
// register use enough to halve throughput.
//
// Lane layout of v_mfma_f64_16x16x4f64 (measured on gfx950):
//   A[i][k] in lane i + 16k, B[k][j] in lane j + 16k,
//   D[i][j] in lane j + 16 (i mod 4), register i / 4.
//
// Workgroups are remapped so that the tiles sharing a row panel of A run
// consecutively on one XCD (the 8 XCDs each have their own L2; hardware hands
// workgroup w to XCD w mod 8).
//
// The left-looking column update (C -= W U^T over the rows below the diagonal
// tile, N = the tile width) has a kernel of its own (gemm_update.hip): all of
// N in one launch and operands staged by direct global-to-LDS loads two K
// slices ahead.
#include <type_traits>

#include "kernels.h"
#include "matern.h"

namespace tlrk {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kXcds = 8;
#ifndef TLRK_GEMM_PAD
#define TLRK_GEMM_PAD 16
#endif

struct GemmArgs {
  int64_t M, N;
  int nseg;
  GemmSeg seg[3];
  int64_t kt[3];       // BK-slices per segment (K padded up to BK)
  int64_t kt_total;
  double* C;
  int64_t ldc;
  GemmEpi ep;
  GemmBatch batch;
  int splitk;
  double* work;
  int64_t gx, gy;      // tile grid
};

// Per-slice column addressing of an operand: element (row gr, slice column kk)
// lives at colbase(kk) + gr (kContig / kPanels) or rowbase(gr) + kk (kContigT).
struct SliceAddr {
  const double* base;
  int64_t ld;
  int64_t col0;   // first column of the slice in the operand's own frame
  int64_t rofs;   // row offset added to gr
};

__device__ inline SliceAddr slice_addr(const Operand& o, int64_t bofs, int64_t kc) {
  SliceAddr s;
  if (o.layout == kPanels) {
    const int64_t c = o.c0 + kc;               // global column of the slice start
    const int64_t p = c / o.nb;                 // one panel holds the whole slice
    s.base = o.base + bofs + panel_offset(o.n, o.nb, p);
    s.ld = o.n - p * o.nb;
    s.col0 = c - p * o.nb;
    s.rofs = o.r0 - p * o.nb;
  } else {
    s.base = o.base + bofs;
    s.ld = o.ld;
    s.col0 = o.c0 + kc;
    s.rofs = o.r0;
  }
  return s;
}

template <int ROWS, int BK, int NT>
__device__ inline void load_slice(const Operand& o, const SliceAddr& sa, int64_t row0, int64_t R, int64_t kc,
                                  int64_t K, double (&v)[ROWS * BK / NT], int tid) {
  constexpr int NE = ROWS * BK / NT;
  if (o.layout == kContigT) {
    const int kk = tid % BK;
    const bool kin = (kc + kk) < K;
#pragma unroll
    for (int p = 0; p < NE; ++p) {
      const int r = tid / BK + (NT / BK) * p;
      const int64_t gr = row0 + r;
      v[p] = (kin && gr < R) ? sa.base[(sa.rofs + gr) * sa.ld + sa.col0 + kk] : 0.0;
    }
  } else {
    const int r = tid % ROWS;
    const int64_t gr = row0 + r;
    const bool rin = gr < R;
#pragma unroll
    for (int p = 0; p < NE; ++p) {
      const int kk = tid / ROWS + (NT / ROWS) * p;
      v[p] = (rin && (kc + kk) < K) ? sa.base[(sa.col0 + kk) * sa.ld + sa.rofs + gr] : 0.0;
    }
  }
}

template <int ROWS, int BK, int PAD, int NT, class ST>
__device__ inline void store_slice(int layout, ST (*s)[ROWS + PAD], const double (&v)[ROWS * BK / NT], int tid) {
  constexpr int NE = ROWS * BK / NT;
  if (layout == kContigT) {
    const int kk = tid % BK;
#pragma unroll
    for (int p = 0; p < NE; ++p) s[kk][tid / BK + (NT / BK) * p] = (ST)v[p];
  } else {
    const int r = tid % ROWS;
#pragma unroll
    for (int p = 0; p < NE; ++p) s[tid / ROWS + (NT / ROWS) * p][r] = (ST)v[p];
  }
}

__device__ inline void epi_store(const GemmEpi& ep, double* C, int64_t ldc, int64_t m, int64_t n, double v,
                                 int64_t grow0) {
  double* c = C + n * ldc + m;
  if (ep.kind == kEpiLinear) {
    double o = ep.alpha * v;
    if (ep.beta != 0.0) o += ep.beta * (*c);
    *c = o;
  } else {
    const double r = loc_dist(ep.mp, ep.x, ep.y, grow0 + m, ep.gcol0 + n);
    double cv, dv;
    if (ep.kind == kEpiGenMinus) {
      matern_eval<false>(ep.mp, r, cv, dv);
      *c = cv - v;
    } else {
      matern_eval<true>(ep.mp, r, cv, dv);
      *c = dv - v;
    }
  }
}

// EPI = 0: linear epilogue only (fewer registers); 1: any epilogue kind.
// DB = 1: two LDS stages, one barrier per K slice.
// TAG 2: the products in FP32 (v_mfma_f32_16x16x4f32, operands rounded to
// FP32 when staged in LDS, FP32 accumulation within the launch), added to the
// FP64 C.  Its output layout differs: D[i][j] in lane j + 16 (i / 4),
// register i mod 4.
template <int BM, int BN, int WM, int WN, int BK, int PAD, int EPI, int DB, int TAG>
__global__ void __launch_bounds__(WM * WN * 64) gemm_kernel(GemmArgs g) {
  constexpr bool F32 = TAG == 2;
  using ST = typename std::conditional<F32, float, double>::type;
  using AV = typename std::conditional<F32, f4, d4>::type;
  constexpr int NT = WM * WN * 64;
  constexpr int TM = BM / WM / 16;
  constexpr int TN = BN / WN / 16;
  constexpr int NS = DB ? 2 : 1;
  __shared__ ST sA[NS][BK][BM + PAD];
  __shared__ ST sB[NS][BK][BN + PAD];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = tid >> 6;
  const int wm = w % WM;
  const int wn = w / WM;

  // XCD-aware remap of the 1-D grid (padded to a multiple of kXcds).
  const bool flat = g.batch.tile_item != nullptr;
  const int64_t total = flat ? g.batch.ntiles : g.gx * g.gy;
  const int64_t per = (total + kXcds - 1) / kXcds;
  const int64_t wid = blockIdx.x;
  const int64_t logical = (wid % kXcds) * per + wid / kXcds;
  if (logical >= total) return;
  int z;
  int64_t tm, tn;
  if (flat) {
    z = g.batch.tile_item[logical];
    const int64_t local = logical - g.batch.tile_first[z];
    const int64_t nz = g.batch.n_of ? g.batch.n_of[z] : g.N;
    const int64_t gyz = (nz + BN - 1) / BN;
    tm = local / gyz;
    tn = local - tm * gyz;
  } else {
    z = blockIdx.y;
    tm = logical / g.gy;
    tn = logical - tm * g.gy;
  }

  int64_t M = g.M, N = g.N;
  int64_t Kb[3] = {g.seg[0].K, g.nseg > 1 ? g.seg[1].K : 0, g.nseg > 2 ? g.seg[2].K : 0};
  int64_t c_off = 0, grow0 = g.ep.grow0;
  int64_t aofs[3] = {0, 0, 0}, bofs[3] = {0, 0, 0};
  int64_t ks = 0, ke = g.kt_total;
  if (g.splitk > 1) {
    const int64_t chunk = (g.kt_total + g.splitk - 1) / g.splitk;
    ks = z * chunk;
    ke = ks + chunk < g.kt_total ? ks + chunk : g.kt_total;
  } else if (g.batch.count > 1 || g.batch.a_off || g.batch.m_of || g.batch.a_off1 || g.batch.a_off2 || g.batch.k_of1 ||
             g.batch.k_of2 || flat) {
    c_off = g.batch.c_off ? g.batch.c_off[z] : z * g.batch.c_bstride;
    grow0 += z * g.ep.grow_bstride;
    for (int s = 0; s < g.nseg; ++s) {
      aofs[s] = z * g.seg[s].a_bstride;
      bofs[s] = z * g.seg[s].b_bstride;
    }
    if (g.batch.a_off) aofs[0] = g.batch.a_off[z];
    if (g.batch.b_off) bofs[0] = g.batch.b_off[z];
    if (g.batch.a_off1) aofs[1] = g.batch.a_off1[z];
    if (g.batch.b_off1) bofs[1] = g.batch.b_off1[z];
    if (g.batch.a_off2) aofs[2] = g.batch.a_off2[z];
    if (g.batch.b_off2) bofs[2] = g.batch.b_off2[z];
    // segments 1 and 2: this item's own K (the rest of the segment reads as zero)
    if (g.batch.k_of1) Kb[1] = g.batch.k_of1[z];
    if (g.batch.k_of2) Kb[2] = g.batch.k_of2[z];
    if (g.batch.m_of) M = g.batch.m_of[z];
    if (g.batch.n_of) N = g.batch.n_of[z];
    if (g.batch.k_of) {
      Kb[0] = g.batch.k_of[z];
      // one segment: the K loop stops at this item's own K
      if (g.nseg == 1) {
        const int64_t kz = (Kb[0] + BK - 1) / BK;
        ke = kz < ke ? kz : ke;
      }
    }
  }
  const int64_t m0 = tm * BM, n0 = tn * BN;
  if (m0 >= M || n0 >= N) return;

  AV acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = AV{0, 0, 0, 0};

  double va[BM * BK / NT], vb[BN * BK / NT];
  auto fetch = [&](int64_t t) {
    int s = 0;
    int64_t tl = t;
    if (g.nseg > 1 && tl >= g.kt[0]) {
      s = 1;
      tl -= g.kt[0];
      if (g.nseg > 2 && tl >= g.kt[1]) {
        s = 2;
        tl -= g.kt[1];
      }
    }
    const GemmSeg& sg = g.seg[s];
    const int64_t kc = tl * BK;
    const SliceAddr saA = slice_addr(sg.A, aofs[s], kc);
    const SliceAddr saB = slice_addr(sg.B, bofs[s], kc);
    load_slice<BM, BK, NT>(sg.A, saA, m0, M, kc, Kb[s], va, tid);
    load_slice<BN, BK, NT>(sg.B, saB, n0, N, kc, Kb[s], vb, tid);
    return s;
  };
  auto compute = [&](int buf) {
#pragma unroll
    for (int k4 = 0; k4 < BK / 4; ++k4) {
      const int kr = k4 * 4 + (lane >> 4);
      ST a[TM], b[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) a[i] = sA[buf][kr][wm * (BM / WM) + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < TN; ++j) b[j] = sB[buf][kr][wn * (BN / WN) + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          if constexpr (F32)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(b[j], a[i], acc[i][j], 0, 0, 0);
          else
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(b[j], a[i], acc[i][j], 0, 0, 0);
        }
    }
  };

  if (ks < ke) {
    int sc = fetch(ks);
    if (DB) {
      store_slice<BM, BK, PAD, NT, ST>(g.seg[sc].A.layout, sA[0], va, tid);
      store_slice<BN, BK, PAD, NT, ST>(g.seg[sc].B.layout, sB[0], vb, tid);
      __syncthreads();
      for (int64_t t = ks; t < ke; ++t) {
        const int cur = (int)((t - ks) & 1);
        const bool more = t + 1 < ke;
        if (more) sc = fetch(t + 1);
        compute(cur);
        if (more) {
          store_slice<BM, BK, PAD, NT, ST>(g.seg[sc].A.layout, sA[cur ^ 1], va, tid);
          store_slice<BN, BK, PAD, NT, ST>(g.seg[sc].B.layout, sB[cur ^ 1], vb, tid);
        }
        __syncthreads();
      }
    } else {
      for (int64_t t = ks; t < ke; ++t) {
        store_slice<BM, BK, PAD, NT, ST>(g.seg[sc].A.layout, sA[0], va, tid);
        store_slice<BN, BK, PAD, NT, ST>(g.seg[sc].B.layout, sB[0], vb, tid);
        __syncthreads();
        if (t + 1 < ke) sc = fetch(t + 1);
        compute(0);
        __syncthreads();
      }
    }
  }

  // epilogue: lane holds rows m = .. + (lane & 15), columns n = .. + (lane >> 4) + 4 r
  // (FP32 products: n = .. + 4 (lane >> 4) + r)
  GemmEpi ep = g.ep;
  if (!EPI) ep.kind = kEpiLinear;
#pragma unroll
  for (int i = 0; i < TM; ++i) {
    const int64_t m = m0 + wm * (BM / WM) + i * 16 + (lane & 15);
#pragma unroll
    for (int j = 0; j < TN; ++j) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t n = n0 + wn * (BN / WN) + j * 16 + (F32 ? 4 * (lane >> 4) + r : (lane >> 4) + 4 * r);
        if (m < M && n < N) {
          const double v = (double)acc[i][j][r];
          if (g.splitk > 1)
            g.work[(int64_t)z * g.M * g.N + n * g.M + m] = v;
          else if (!EPI) {
            double* c = g.C + c_off + n * g.ldc + m;
            double o = ep.alpha * v;
            if (ep.beta != 0.0) o += ep.beta * (*c);
            *c = o;
          } else
            epi_store(ep, g.C + c_off, g.ldc, m, n, v, grow0);
        }
      }
    }
  }
}

template <int TAG>
__global__ void __launch_bounds__(256) splitk_reduce_kernel(GemmArgs g) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= g.M * g.N) return;
  const int64_t n = idx / g.M;
  const int64_t m = idx - n * g.M;
  double v = 0.0;
  for (int z = 0; z < g.splitk; ++z) v += g.work[(int64_t)z * g.M * g.N + idx];
  epi_store(g.ep, g.C, g.ldc, m, n, v, g.ep.grow0);
}

template <int BM, int BN, int WM, int WN, int BK = 32, int PAD = TLRK_GEMM_PAD, int EPI = 1, int DB = 0,
          int TAG = 0>
static hipError_t run(GemmArgs& g, int zdim, hipStream_t s) {
  g.kt_total = 0;
  for (int i = 0; i < g.nseg; ++i) {
    g.kt[i] = (g.seg[i].K + BK - 1) / BK;
    g.kt_total += g.kt[i];
  }
  for (int i = 0; i < g.nseg; ++i)
    for (const Operand* o : {&g.seg[i].A, &g.seg[i].B})
      if (o->layout == kPanels && (o->nb % BK != 0 || o->c0 % BK != 0)) return hipErrorInvalidValue;
  g.gx = (g.M + BM - 1) / BM;
  g.gy = (g.N + BN - 1) / BN;
  if (g.batch.tile_item) zdim = 1;
  const int64_t total = g.batch.tile_item ? g.batch.ntiles : g.gx * g.gy;
  const int64_t grid = ((total + kXcds - 1) / kXcds) * kXcds;
  if (grid > 0x7fffffff || zdim > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL((gemm_kernel<BM, BN, WM, WN, BK, PAD, EPI, DB, TAG>), dim3((unsigned)grid, (unsigned)zdim),
                     dim3(WM * WN * 64), 0, s, g);
  return hipGetLastError();
}

template <int TAG>
static hipError_t launch_gemm_t(int64_t M, int64_t N, int nseg, const GemmSeg* segs, double* C, int64_t ldc,
                                const GemmEpi& ep_in, const GemmBatch* batch, int splitk, double* work,
                                hipStream_t s, int tile_m, int tile_n) {
  if (M < 0 || N < 0 || nseg < 1 || nseg > 3 || splitk < 1) return hipErrorInvalidValue;
  if (M == 0 || N == 0) return hipSuccess;
  GemmEpi ep = ep_in;
  if (ep.kind != kEpiLinear) {
    // generation first (C = Matern or dMatern/dbeta entries), then C -= A B^T:
    // keeping the Matern code out of the MFMA kernel keeps its register
    // allocation and schedule lean
    if (batch && (batch->count > 1 || batch->a_off || batch->m_of)) return hipErrorInvalidValue;
    hipError_t e = launch_matern_block(ep.mp, ep.x, ep.y, ep.grow0, M, ep.gcol0, N, C, ldc, ep.kind == kEpiDGenMinus, s);
    if (e != hipSuccess) return e;
    ep.kind = kEpiLinear;
    ep.alpha = -1.0;
    ep.beta = 1.0;
  }
  GemmArgs g{};
  g.M = M;
  g.N = N;
  g.nseg = nseg;
  g.kt_total = 0;
  bool panels = false, bk32 = true;
  for (int i = 0; i < nseg; ++i) {
    g.seg[i] = segs[i];
    if (segs[i].K < 0) return hipErrorInvalidValue;
    for (const Operand* o : {&segs[i].A, &segs[i].B})
      if (o->layout == kPanels) {
        panels = true;
        if (o->nb % 16 != 0 || o->c0 % 16 != 0) return hipErrorInvalidValue;
        if (o->nb % 32 != 0 || o->c0 % 32 != 0) bk32 = false;
      }
    g.kt[i] = (segs[i].K + 15) / 16;
    g.kt_total += g.kt[i];
  }
  if (g.kt_total == 0 && ep.alpha == -1.0 && ep.beta == 1.0) return hipSuccess;  // C already final
  g.C = C;
  g.ldc = ldc;
  g.ep = ep;
  if (batch) g.batch = *batch; else { g.batch = GemmBatch{}; g.batch.count = 1; }
  if (g.batch.count < 1) return hipErrorInvalidValue;
  if (splitk > 1 && (g.batch.count > 1 || work == nullptr)) return hipErrorInvalidValue;
  if (splitk > g.kt_total) splitk = g.kt_total > 0 ? (int)g.kt_total : 1;
  g.splitk = splitk;
  g.work = work;
  const int zdim = splitk > 1 ? splitk : g.batch.count;
  hipError_t e;
  if (g.batch.tile_item) {   // the tile list was built for exactly these tile sizes
    const int key = tile_m * 1000 + tile_n;
    if (key != 32032 && key != 32064 && key != 32128 && key != 64032 && key != 64064 && key != 64128 &&
        key != 128032 && key != 128064 && key != 128128)
      return hipErrorInvalidValue;
  }
  if (tile_m || tile_n) {
    // hinted small tiles (batched low-rank products): four waves, one LDS stage
    const int bm = tile_m ? tile_m : 128, bn = tile_n ? tile_n : 128;
    switch (bm * 1000 + bn) {
      case 32032: e = run<32, 32, 2, 2, 32, 4, 0, 0, TAG>(g, zdim, s); break;
      case 32064: e = run<32, 64, 2, 2, 32, 4, 0, 0, TAG>(g, zdim, s); break;
      case 32128: e = run<32, 128, 2, 2, 32, 4, 0, 0, TAG>(g, zdim, s); break;
      case 64032: e = run<64, 32, 2, 2, 32, 4, 0, 0, TAG>(g, zdim, s); break;
      case 64064: e = run<64, 64, 2, 2, 32, 4, 0, 0, TAG>(g, zdim, s); break;
      case 64128: e = run<64, 128, 2, 2, 32, 4, 0, 0, TAG>(g, zdim, s); break;
      case 128032: e = run<128, 32, 2, 2, 32, 4, 0, 0, TAG>(g, zdim, s); break;
      case 128064: e = run<128, 64, 2, 2, 32, 4, 0, 0, TAG>(g, zdim, s); break;
      default: e = run<128, 128, 2, 4, 32, 4, 0, 1, TAG>(g, zdim, s); break;
    }
  } else if (panels && !bk32) {
    e = run<128, 128, 2, 4, 16, 4, 0, 1, TAG>(g, zdim, s);
  } else if (M >= 2048 && N >= 1024) {
    e = run<256, 128, 4, 2, 16, 4, 0, 1, TAG>(g, zdim, s);
  } else if (N <= 32) {
    e = run<128, 32, 2, 2, 32, 4, 0, 0, TAG>(g, zdim, s);
  } else if (N <= 64) {
    e = run<128, 64, 2, 2, 32, 4, 0, 1, TAG>(g, zdim, s);
  } else if (M <= 32) {
    e = run<32, 128, 2, 2, 32, 4, 0, 0, TAG>(g, zdim, s);
  } else if (M <= 64) {
    e = run<64, 128, 2, 2, 32, 4, 0, 1, TAG>(g, zdim, s);
  } else if (TAG == 1 && nseg == 1 && splitk == 1 && g.batch.count == 1 && !g.batch.m_of && !g.batch.a_off &&
             launch_gemm_update(g.seg[0], M, N, C, ldc, ep, s, &e)) {
    return e;
  } else if (TAG != 0 && splitk == 1 && g.batch.count == 1 && !g.batch.m_of && N >= 256 && N % 256 <= 64) {
    // column update: 128 x 256 tiles (wave tile 64 x 64) over the first 256 q
    // columns: each W slice feeds twice the MFMAs of a 128 x 128 tile, and the
    // W panel is streamed by half as many tile columns; the rest as below
    const int64_t n1 = N - N % 256;
    g.N = n1;
    e = run<128, 256, 2, 4, 16, 4, 0, 1, TAG>(g, zdim, s);
    if (e != hipSuccess || n1 == N) return e;
    GemmArgs g2 = g;
    g2.N = N - n1;
    for (int i = 0; i < g2.nseg; ++i) g2.seg[i].B.r0 += n1;
    g2.C = C + n1 * ldc;
    g2.ep.gcol0 += n1;
    if (N - n1 <= 32)
      e = run<128, 32, 2, 2, 32, 4, 0, 0, TAG>(g2, zdim, s);
    else
      e = run<128, 64, 2, 2, 32, 4, 0, 1, TAG>(g2, zdim, s);
  } else if (splitk == 1 && g.batch.count == 1 && !g.batch.m_of && N % 128 != 0 && N % 128 <= 64) {
    // N = 128 q + r (r <= 64): 128 x 128 tiles over the first 128 q columns,
    // 128 x r-wide tiles over the rest, instead of a mostly idle last tile column
    const int64_t n1 = N - N % 128;
    g.N = n1;
    e = run<128, 128, 2, 4, 32, 4, 0, 1, TAG>(g, zdim, s);
    if (e != hipSuccess) return e;
    GemmArgs g2 = g;
    g2.N = N - n1;
    for (int i = 0; i < g2.nseg; ++i) g2.seg[i].B.r0 += n1;
    g2.C = C + n1 * ldc;
    g2.ep.gcol0 += n1;
    if (N - n1 <= 32)
      e = run<128, 32, 2, 2, 32, 4, 0, 0, TAG>(g2, zdim, s);
    else
      e = run<128, 64, 2, 2, 32, 4, 0, 1, TAG>(g2, zdim, s);
  } else {
    e = run<128, 128, 2, 4, 32, 4, 0, 1, TAG>(g, zdim, s);
  }
  if (e != hipSuccess || splitk == 1) return e;
  const int64_t tot = M * N;
  hipLaunchKernelGGL(splitk_reduce_kernel<TAG>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, g);
  return hipGetLastError();
}

hipError_t launch_gemm(int64_t M, int64_t N, int nseg, const GemmSeg* segs, double* C, int64_t ldc,
                       const GemmEpi& ep, const GemmBatch* batch, int splitk, double* work, hipStream_t s,
                       int tile_m, int tile_n, int tag) {
  if (tag == 1) return launch_gemm_t<1>(M, N, nseg, segs, C, ldc, ep, batch, splitk, work, s, tile_m, tile_n);
  if (tag == 2) return launch_gemm_t<2>(M, N, nseg, segs, C, ldc, ep, batch, splitk, work, s, tile_m, tile_n);
  return launch_gemm_t<0>(M, N, nseg, segs, C, ldc, ep, batch, splitk, work, s, tile_m, tile_n);
}

// ---------------------------------------------------------------------------
// Batched products with a small inner dimension, C_p = alpha A_p B_p + beta
// C_p (A_p: m_p x k_p, B_p: k_p x n_p -- or its transpose stored, btrans --
// column-major at element offsets a_off[p], b_off[p], c_off[p]).  In the
// column update these are W_ik = U_ik X_ik: 800 rows, k and n ranks of a few
// tens, thousands of pairs; in the tangent's correction dC_ij -= U_ij P_ij^T
// (n = 800).  Memory-bound: A is streamed
// (once per 16 columns of C, re-reads hit L2), B is staged in LDS 16
// columns at a time and read as broadcasts, each thread owns one row of C.
// Workgroup (p, y, z) covers rows [256 y, 256 y + 256) and columns
// [kThinGroup z, kThinGroup (z + 1)) of pair p.
// ---------------------------------------------------------------------------
namespace {
constexpr int kThinRows = 256;
constexpr int kThinCols = 16;
constexpr int kThinGroup = 32;   // columns per workgroup
}  // namespace

__global__ void __launch_bounds__(kThinRows) thin_gemm_kernel(const double* __restrict__ A, int64_t lda,
                                                              const double* __restrict__ B, int64_t ldb,
                                                              double* __restrict__ C, int64_t ldc,
                                                              const int* __restrict__ m_of,
                                                              const int* __restrict__ n_of,
                                                              const int* __restrict__ k_of,
                                                              const int64_t* __restrict__ a_off,
                                                              const int64_t* __restrict__ b_off,
                                                              const int64_t* __restrict__ c_off, double alpha,
                                                              double beta, int btrans) {
  extern __shared__ double xs[];   // [k][kThinCols]
  const int p = blockIdx.x;
  const int m = m_of[p], n = n_of[p], k = k_of[p];
  const int r0 = blockIdx.y * kThinRows;
  if (r0 >= m || n <= 0) return;   // uniform over the workgroup
  const int r = r0 + threadIdx.x;
  const double* a = A + a_off[p];
  const double* b = B + b_off[p];
  double* c = C + c_off[p];
  const int n1 = (n < (int)(blockIdx.z + 1) * kThinGroup) ? n : (int)(blockIdx.z + 1) * kThinGroup;
  for (int n0 = blockIdx.z * kThinGroup; n0 < n1; n0 += kThinCols) {
    const int nc = (n1 - n0 < kThinCols) ? n1 - n0 : kThinCols;
    __syncthreads();   // the previous slice has been read
    if (btrans) {   // B^T stored: element (t, q) at b[q + t ldb]
      for (int e = threadIdx.x; e < k * kThinCols; e += kThinRows) {
        const int t = e / kThinCols, q = e - t * kThinCols;
        xs[e] = (q < nc) ? b[(n0 + q) + (int64_t)t * ldb] : 0.0;
      }
    } else {
      for (int e = threadIdx.x; e < k * kThinCols; e += kThinRows) {
        const int q = e / k, t = e - q * k;   // consecutive threads: consecutive rows of B
        xs[t * kThinCols + q] = (q < nc) ? b[t + (int64_t)(n0 + q) * ldb] : 0.0;
      }
    }
    __syncthreads();
    if (r < m) {
      double acc[kThinCols];
#pragma unroll
      for (int q = 0; q < kThinCols; ++q) acc[q] = 0.0;
      const double* ar = a + r;
#pragma unroll 4
      for (int t = 0; t < k; ++t) {
        const double u = ar[(int64_t)t * lda];
        const double* xt = xs + t * kThinCols;
#pragma unroll
        for (int q = 0; q < kThinCols; ++q) acc[q] += u * xt[q];
      }
#pragma unroll
      for (int q = 0; q < kThinCols; ++q)
        if (q < nc) {
          double* cq = c + r + (int64_t)(n0 + q) * ldc;
          *cq = beta == 0.0 ? alpha * acc[q] : alpha * acc[q] + beta * *cq;
        }
    }
  }
}

hipError_t launch_thin_gemm(const double* A, int64_t lda, const double* B, int64_t ldb, double* C, int64_t ldc,
                            const GemmBatch& batch, int maxm, int maxk, int maxn, hipStream_t s, double alpha,
                            double beta, bool btrans) {
  if (batch.count <= 0 || maxm <= 0) return hipSuccess;
  if (maxk < 0 || maxk > kThinMaxK || !batch.m_of || !batch.n_of || !batch.k_of || !batch.a_off ||
      !batch.b_off || !batch.c_off)
    return hipErrorInvalidValue;
  const size_t lds = (size_t)(maxk > 0 ? maxk : 1) * kThinCols * sizeof(double);
  const unsigned groups = (unsigned)((maxn + kThinGroup - 1) / kThinGroup);
  hipLaunchKernelGGL(thin_gemm_kernel,
                     dim3((unsigned)batch.count, (unsigned)((maxm + kThinRows - 1) / kThinRows), groups > 0 ? groups : 1),
                     dim3(kThinRows), lds, s, A, lda, B, ldb, C, ldc, batch.m_of, batch.n_of, batch.k_of,
                     batch.a_off, batch.b_off, batch.c_off, alpha, beta, btrans ? 1 : 0);
  return hipGetLastError();
}

}  // namespace tlrk
