// Adaptive cross approximation of Matérn tiles fused with their generation (aca.hip).
#pragma once
#include "common.h"

namespace tlrk {

// One tile: rows r0 .. r0 + m - 1 and columns c0 .. c0 + n - 1 of Sigma
// (global point indices), m, n <= 1024.  Output U (m x k, column-major, ld)
// and V (n x k, ld) with tile ~ U V^T, k <= kmax columns written, and
// *rank = k, or kmax + 1 when kmax steps did not reach the stopping rule.
struct AcaTask {
  int64_t r0, c0;
  int m, n;
  double* U;
  double* V;
  int64_t ld;
  int* rank;
};

hipError_t launch_aca(const MaternParams& p, const double* x, const double* y, const AcaTask* d_tasks, int count,
                      int kmax, double tau, hipStream_t s);

}  // namespace tlrk
