// Gradient building blocks (grad.hip).
#pragma once
#include "common.h"

namespace tlrk {

// number of workgroups (and partial sums) of launch_pair_quad
int64_t pair_quad_blocks(int64_t n);
// *out = a^T dSigma/dbeta a over all n x n pairs (partial: pair_quad_blocks(n) doubles)
hipError_t launch_pair_quad(const MaternParams& p, const double* x, const double* y, const double* a, int64_t n,
                            double* partial, double* out, hipStream_t s);
// M <- Phi(M) (tril, halved diagonal), *trace_out = tr(M)
hipError_t launch_phi_trace(double* M, int64_t ld, int64_t m, double* trace_out, hipStream_t s);

}  // namespace tlrk
