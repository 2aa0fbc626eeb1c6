// TLR solve building blocks (solve.hip).
#pragma once
#include "common.h"

namespace tlrk {

// Apply the strictly-lower tiles of one column (forward) or one row
// (backward) of a TLR factor held in fixed-size slots:
//   forward, column j:  out_i += scale U_ij (V_ij^T v_j)   for i = j+1 .. nt-1
//   backward, row i:    out_j += scale V_ij (U_ij^T v_i)   for j = 0 .. i-1
struct LowRankApply {
  const double* arena; // U_ij = arena + uoff[i*nt+j], V_ij = arena + voff[...], both ld nb
  const int64_t* uoff;
  const int64_t* voff;
  const int* ranks;    // device rank table, ranks[i * nt + j]
  int64_t n;
  int nb, nt;
  int fixed;
  int forward;
  const double* v;     // full-length vector read
  double* out;         // full-length vector updated
  double scale;        // out += scale * (product); the solves use -1
  double* tws;         // workspace: kLrMaxRank doubles per tile of the launch (t = B^T v)
};
constexpr int kLrMaxRank = 1024;   // ranks (and dense tiles' nb) up to this

// kmax: the largest rank among the launch's tiles (<= kLrMaxRank); a.tws holds
// count * kLrMaxRank doubles.
hipError_t launch_lowrank_apply(const LowRankApply& a, int count, hipStream_t s, int kmax);

}  // namespace tlrk
