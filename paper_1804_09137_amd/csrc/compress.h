// Compression building blocks (compress.hip).
#pragma once
#include "common.h"

namespace tlrk {

constexpr int kQrMaxRows = 1024;   // tile rows (nb) limit of qrcp_kernel
constexpr int kQrMaxCols = 512;    // sketch / projection width limit

// Column-pivoted Householder QR of the m x q matrix Y (ld), in place, stopped
// at the first step t where the Frobenius norm of the unreduced block
// Y[t:, t:] is <= tol or t == max_rank.
struct QrcpTask {
  double* Y;
  int64_t ldy;
  int m, q;
  double tol;
  int max_rank;
  int min_tail;    // flag = 1 when q - rank < min_tail (sketch too narrow)
  double* Q;       // optional: explicit m x rank orthonormal factor (ldq)
  int64_t ldq;
  double* Z;       // optional: q x rank matrix Z[perm[c], r] = R[r, c] (ldz)
  int64_t ldz;
  int* rank;
  int* flag;
  int upper;       // qrcp_reg: read only the upper triangle of Y (zeros below)
  double* W;       // qrcp_reg: m x rank workspace for the reflectors (ldw)
  int64_t ldw;
  double* tau;     // qrcp_reg, optional: the rank reflector scalars (with W, the
                   // input of wy_build and hqr_apply when Q is not formed here)
};

// On-chip pivoted QR (qrcp_reg_kernel): all in registers up to kRegQrMax
// rows and columns, registers plus LDS up to kRegQrBig.
constexpr int kRegQrMax = 192;
constexpr int kRegQrBig = 224;

// Blocked Householder QR (hqr_factor_kernel) of the m x s matrix A (lda), in
// place, m <= kQrMaxRows, s <= kQrMaxCols; and the application of its Q
// (hqr_apply_kernel) to X (m x kx, ldx).
struct HqrTask {
  double* A;
  int64_t lda;
  int m, s;
  double* T;        // ceil(min(m, s) / 16) compact-WY factors, 256 doubles each
  double tol;       // factor: > 0 selects the range rank (rank, flag)
  int min_tail;
  int* rank;
  int* flag;
  double* X;        // apply: X <- Q X
  int64_t ldx;
  int kx;
  int xrows;        // apply (identity == 0): rows >= xrows of X are cleared first
  int identity;     // apply: X starts as [I_kx; 0]
  const double* tau;   // wy_build: the s reflector scalars
  // factor, trunc != 0 (with tol > 0): rank = the smallest k with
  // ||R[k:, k:]||_F <= tol instead of the range rank, flag = 0, and the rows
  // of R written out transposed: Z[c + r ldz] = R[r, c] for c >= r, 0 for
  // c < r, over r < min(min(m, s), zcap) and c < s.
  int trunc;
  int zcap;
  double* Z;
  int64_t ldz;
};

hipError_t launch_qrcp(const QrcpTask* d_tasks, int count, hipStream_t s, int max_m = kQrMaxRows);
hipError_t launch_qrcp_reg(const QrcpTask* d_tasks, int count, hipStream_t s);
hipError_t launch_hqr_factor(const HqrTask* d_tasks, int count, hipStream_t s);
// X columns are split over workgroups kApplyCols at a time: max_kx must be
// at least every task's kx (columns beyond the split it covers are left
// untouched).
constexpr int kApplyCols = 16;
// With d_items, one workgroup per (task, chunk) pair listed there (2 ints
// each, nitems pairs; the order is the dispatch order) instead of the full
// count x chunks grid.
hipError_t launch_hqr_apply(const HqrTask* d_tasks, int count, hipStream_t s, int max_kx,
                            const int* d_items = nullptr, int nitems = 0);
// The compact-WY factors T (per 16 reflectors, the layout hqr_factor writes)
// of s Householder vectors stored as hqr_factor stores them (A, lda, m rows,
// unit diagonal implied) with scalars tau; max_s >= every task's min(m, s).
hipError_t launch_wy_build(const HqrTask* d_tasks, int count, hipStream_t s, int max_s);
hipError_t launch_copy_upper(const double* src, int64_t sld, const int64_t* soff, double* dst, int64_t dld,
                             const int64_t* doff, const int* nn, int nmax, int count, hipStream_t s);
hipError_t launch_gaussian(double* out, int64_t count, uint32_t seed, hipStream_t s);
hipError_t launch_batched_copy(const double* src, int64_t sld, const int64_t* soff, double* dst, int64_t dld,
                               const int64_t* doff, const int* mrows, const int* kcols, int64_t max_elems,
                               int count, hipStream_t s);

}  // namespace tlrk
