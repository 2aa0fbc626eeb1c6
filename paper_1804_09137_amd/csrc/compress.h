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
};

hipError_t launch_qrcp(const QrcpTask* d_tasks, int count, hipStream_t s);
hipError_t launch_gaussian(double* out, int64_t count, uint32_t seed, hipStream_t s);
hipError_t launch_batched_copy(const double* src, int64_t sld, const int64_t* soff, double* dst, int64_t dld,
                               const int64_t* doff, const int* mrows, const int* kcols, int64_t max_elems,
                               int count, hipStream_t s);

}  // namespace tlrk
