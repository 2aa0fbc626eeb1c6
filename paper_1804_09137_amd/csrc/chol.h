// Dense tile building blocks (chol.hip) and the blocked tile factorisation.
#pragma once
#include "common.h"

namespace tlrk {

hipError_t launch_potrf_small(double* A, int64_t lda, int w, double* Inv, int64_t ldi,
                              unsigned long long* info, int64_t row0, hipStream_t s);
hipError_t launch_zero_upper(double* A, int64_t lda, int64_t m, hipStream_t s);
hipError_t launch_copy_block(const double* in, int64_t ldi, double* out, int64_t ldo, int64_t m, int64_t ncol,
                             hipStream_t s);
hipError_t launch_logdiag(const double* A, int64_t lda, int64_t m, double* out, hipStream_t s);
hipError_t launch_gemv_n(const double* A, int64_t lda, int64_t m, int64_t k, const double* x, double alpha,
                         double beta, double* y, hipStream_t s);
hipError_t launch_gemv_t(const double* A, int64_t lda, int64_t m, int64_t k, const double* x, double alpha,
                         double beta, double* y, hipStream_t s);
hipError_t launch_fill(double* A, int64_t lda, int64_t m, int64_t ncol, double value, hipStream_t s);
hipError_t launch_identity(double* A, int64_t lda, int64_t m, hipStream_t s);
// *acc += sum (A - B)^2 over the m x ncol block (B null: sum A^2); acc is device memory
hipError_t launch_sqdiff_acc(const double* A, int64_t lda, const double* B, int64_t ldb, int64_t m, int64_t ncol,
                             double* acc, hipStream_t s);
hipError_t launch_dot(const double* a, const double* b, int64_t m, double* out, hipStream_t s);
// n ints src -> dst and (w_src non-null) one word w_src -> w_dst, then *flag =
// seq (system-scope release); dst, w_dst and flag are fine-grained host memory
hipError_t launch_publish(const int* src, int n, int* dst, const unsigned long long* w_src, unsigned long long* w_dst,
                          unsigned* flag, unsigned seq, hipStream_t s);

// Lower Cholesky of the m x m tile T (column-major, ld) in place, blocked
// left-looking with 64-wide blocks; writes the inverse factor to Inv (ldi) and
// zeroes the strict upper parts of both.  work holds >= 64 * m doubles.
hipError_t tile_potrf_inv(double* T, int64_t ld, int64_t m, double* Inv, int64_t ldi, unsigned long long* info,
                          int64_t row0, double* work, hipStream_t s);

}  // namespace tlrk
