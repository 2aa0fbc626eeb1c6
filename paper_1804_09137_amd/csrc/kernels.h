// Launch wrappers of the HIP kernels (host-callable, stream-ordered).
#pragma once
#include "common.h"

namespace tlrk {

// ---------------------------------------------------------------- matern.hip
hipError_t launch_matern_block(const MaternParams& p, const double* x, const double* y, int64_t r0, int64_t m,
                               int64_t c0, int64_t ncol, double* out, int64_t ld, bool deriv, hipStream_t s);

// ------------------------------------------------------------------ gemm.hip
// C[M x N] = epilogue( sum_s A_s[M x K_s] * B_s[N x K_s]^T ), FP64 MFMA, up to 3 segments.
// Operand layouts: kContig (rows contiguous), kContigT (columns contiguous,
// i.e. X[r, c] = base[(r0 + r) * ld + c0 + c]) and kPanels.
enum : int { kContigT = 2 };

enum EpiKind : int {
  kEpiLinear = 0,    // C = alpha * acc + beta * C_in
  kEpiGenMinus = 1,  // C = Matérn(theta)(rows, cols) - acc
  kEpiDGenMinus = 2, // C = dMatérn/dbeta(rows, cols) - acc
};

struct GemmSeg {
  Operand A, B;
  int64_t K;
  int64_t a_bstride, b_bstride;  // element offset of batch z
};

struct GemmEpi {
  int kind;
  double alpha, beta;
  MaternParams mp;
  const double* x;  // locations (kEpiGen*)
  const double* y;
  int64_t grow0, gcol0;     // global point index of output row 0 / col 0
  int64_t grow_bstride;     // per-batch shift of grow0
};

struct GemmBatch {
  int count;                 // >= 1
  int64_t c_bstride;         // element offset of batch z in C
  const int* m_of;           // optional device arrays: per-batch M, N, K (<= the launch M, N, K)
  const int* n_of;
  const int* k_of;
  const int64_t* a_off;      // optional device arrays: per-batch element offsets of
  const int64_t* b_off;      //   segment 0's A and B and of C (replace the strides)
  const int64_t* c_off;
  // optional flat tile list (hinted tile sizes only): workgroup w computes
  // tile w - tile_first[z] of batch z = tile_item[w]; ntiles in all.  Without
  // it every batch gets the launch maximum's tile grid, most of it empty when
  // the per-batch sizes vary.
  const int* tile_item;
  const int* tile_first;
  int64_t ntiles;
  // optional device arrays: per-batch element offsets of segment 1's A and B
  const int64_t* a_off1;
  const int64_t* b_off1;
  // optional device arrays: per-batch element offsets of segment 2's A and B,
  // and per-batch K of segments 1 and 2 (at most the segment's K; the rest of
  // the segment reads as zero)
  const int64_t* a_off2;
  const int64_t* b_off2;
  const int* k_of1;
  const int* k_of2;
};

// Returns hipErrorInvalidValue on bad shapes.  work (may be null) must hold
// splitk * M * N doubles when splitk > 1 (batch count must be 1 then).
// tile_m / tile_n (32, 64 or 128; 0 = by M and N) choose the workgroup tile:
// batched calls whose per-batch sizes are far below the launch maxima use
// small tiles so that the workgroups of small problems stay short.
// tag 1 launches separately named kernel instances (same code), so that a
// kernel trace tells the left-looking column-update GEMMs apart; tag 2 is the
// same with the products in FP32 (operands rounded to FP32, FP32 MFMA and
// accumulation within the launch, result added to the FP64 C).
hipError_t launch_gemm(int64_t M, int64_t N, int nseg, const GemmSeg* segs, double* C, int64_t ldc,
                       const GemmEpi& ep, const GemmBatch* batch, int splitk, double* work, hipStream_t s,
                       int tile_m = 0, int tile_n = 0, int tag = 0);

// ----------------------------------------------------------- gemm_update.hip
// C = alpha A B^T + beta C (ep linear) by the column-update kernel when the call
// fits it: one segment, both operands kContig with even leading dimensions
// and 16-byte aligned origins, N = 256 q or 256 q + 32.  Returns false (and
// launches nothing) otherwise; else *err is the launch status.
bool launch_gemm_update(const GemmSeg& sg, int64_t M, int64_t N, double* C, int64_t ldc, const GemmEpi& ep,
                        hipStream_t s, hipError_t* err);

// C_p = alpha A_p B_p + beta C_p for a batch of products with a small inner
// dimension (k_p <= kThinMaxK): batch supplies m_of, n_of, k_of and the
// element offsets a_off, b_off, c_off (device arrays, all required); A, B and
// C are column-major with leading dimensions lda, ldb, ldc; btrans: B_p^T is
// stored instead (element (t, q) of B_p at b[q + t ldb]).  maxm, maxk, maxn:
// the largest m_p, k_p and n_p.  Returns hipErrorInvalidValue for maxk >
// kThinMaxK.
constexpr int kThinMaxK = 512;   // B slice in LDS: kThinMaxK x 16 doubles (64 KB)
hipError_t launch_thin_gemm(const double* A, int64_t lda, const double* B, int64_t ldb, double* C, int64_t ldc,
                            const GemmBatch& batch, int maxm, int maxk, int maxn, hipStream_t s,
                            double alpha = 1.0, double beta = 0.0, bool btrans = false);

}  // namespace tlrk
