// Shared device/host definitions for the TLR Matérn log-likelihood library.
// gfx950 (CDNA4) only: 64-lane wavefronts, FP64 MFMA 16x16x4.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>

namespace tlrk {

constexpr int kWave = 64;

// ----------------------------------------------------------------------------
// Matérn covariance parameters, Eq. (MaternCov) of Section IV:
//   C(r) = sigma2 / (2^(nu-1) Gamma(nu)) * u^nu K_nu(u),  u = r / beta.
// Everything that depends only on theta is computed once on the host.
// ----------------------------------------------------------------------------
enum MaternKind : int { kNuHalf = 0, kNuThreeHalves = 1, kNuFiveHalves = 2, kNuGeneral = 3 };

// Distance between locations (Section IV): Euclidean in the plane, or the
// great-circle distance of Eq. (gcd) (haversine formula) for (longitude,
// latitude) in degrees on a sphere of radius `radius`.
enum Metric : int { kMetricEuclid = 0, kMetricGreatCircle = 1 };

constexpr int kTemmeTerms = 40;     // Temme series length cap (x <= 2 needs < 20)
constexpr int kTrapBuckets = 9;     // trapezoid buckets in x (x > 2)
constexpr int kTrapTerms = 32;      // nodes per bucket cap (needs <= 27)

// Device-resident tables for general nu; laid out as doubles:
//   temme[4][kTemmeTerms]: 1/(k-mu), 1/(k+mu), 1/(k^2-mu^2), 1/k  for k = 1..kTemmeTerms
//   trap[kTrapBuckets][3][kTrapTerms]: cosh(t_k)-1, cosh(nu t_k), cosh((nu-1) t_k), t_k = k h_b
//   dnu[3][kDnuNodes]: cosh(t_k) - 1, cosh(nu t_k), t_k sinh(nu t_k), t_k = k kDnuH
//   (every nu: the derivative in nu)
constexpr int kDnuNodes = 128;
constexpr double kDnuH = 0.25;
constexpr int kTabTemme = 0;
constexpr int kTabTrap = 4 * kTemmeTerms;
constexpr int kTabDnu = kTabTrap + kTrapBuckets * 3 * kTrapTerms;
constexpr int kTabSize = kTabDnu + 3 * kDnuNodes;

// Which derivative matern_eval<true> returns: dC/dbeta or dC/dnu.
enum MaternDeriv : int { kDerivBeta = 1, kDerivNu = 2 };

struct MaternParams {
  double sigma2, beta, inv_beta, nu;
  double norm;          // sigma2 / (2^(nu-1) Gamma(nu))
  int kind;             // MaternKind
  // general nu: Temme pair order mu in [-1/2, 1/2]
  int nrec;             // forward recurrence steps after the Temme/trapezoid pair
  int pair_swapped;     // 1: the (mu, mu+1) pair is (K_nu, K_{nu-1}) (nu <= 1/2)
  double mu;
  double G1, G2;        // Temme's Gamma_1(mu), Gamma_2(mu)
  double rgp, rgm;      // 1/Gamma(1+mu), 1/Gamma(1-mu)
  double fac;           // mu pi / sin(mu pi)
  double trap_h[kTrapBuckets];
  int trap_n[kTrapBuckets];
  const double* tab;    // device tables (kTabSize doubles), general nu only
  int metric;           // Metric
  double radius;        // kMetricGreatCircle: sphere radius (distance unit)
  int dparam;           // MaternDeriv: the parameter of the derivative (kDerivBeta by default)
  double psi;           // digamma(nu), for dC/dnu
};

// Host: fill p for theta = (sigma2, beta, nu); writes the kTabSize-double table
// into host_tab (caller copies it to p.tab's device buffer).  Returns false if
// theta is not finite and positive.
bool matern_setup(double sigma2, double beta, double nu, MaternParams* p, double* host_tab);

// ----------------------------------------------------------------------------
// Operand addressing for the FP64 MFMA GEMM.  An operand is an R x K matrix
// (rows = output rows or columns, K = contraction) read as X[r, c].
//   kContig: X[r, c] = base[(c0 + c) * ld + r0 + r]
//   kPanels: lower-panel storage of an n x n lower-triangular matrix with
//            column panels of width nb; panel p holds rows p*nb .. n-1 of
//            columns p*nb .. p*nb+nb-1, column-major with ld = n - p*nb.
//            X[r, c] is global element (r0 + r, c0 + c).
// ----------------------------------------------------------------------------
enum Layout : int { kContig = 0, kPanels = 1 };

struct Operand {
  const double* base;
  int64_t ld;       // kContig leading dimension
  int64_t r0, c0;   // origin
  int64_t n;        // kPanels: matrix order
  int32_t nb;       // kPanels: panel width
  int32_t layout;
};

__host__ __device__ inline int64_t panel_offset(int64_t n, int64_t nb, int64_t p) {
  // sum_{q < p} (n - q nb) nb
  return p * n * nb - nb * nb * (p * (p - 1) / 2);
}

// Address of global element (r, c), r >= c's panel start, in lower-panel storage.
__host__ __device__ inline int64_t panel_index(int64_t n, int64_t nb, int64_t r, int64_t c) {
  int64_t p = c / nb;
  int64_t cc = c - p * nb;
  return panel_offset(n, nb, p) + cc * (n - p * nb) + (r - p * nb);
}

inline int64_t panels_size(int64_t n, int64_t nb) {
  int64_t nt = (n + nb - 1) / nb;
  return panel_offset(n, nb, nt - 1) + (n - (nt - 1) * nb) * (n - (nt - 1) * nb);
}

}  // namespace tlrk
