// Matérn covariance generation (Section IV, Eq. (MaternCov)): host-side
// parameter setup and the standalone block generator kernel.
#include "matern.h"
#include "kernels.h"

#include <cmath>

namespace tlrk {

namespace {
// Taylor coefficients of 1/Gamma(1+z) = sum_k a_k z^k (cf. Abramowitz & Stegun
// 6.1.34, shifted by one), evaluated with mpmath at 40 digits by
// paper_1804_09137_amd/csrc/gen_rgamma_coeffs.py.
const double kRGamma[26] = {
    1.0,
    0.57721566490153286061,
    -0.65587807152025388108,
    -0.042002635034095235529,
    0.1665386113822914895,
    -0.042197734555544336748,
    -0.0096219715278769735621,
    0.0072189432466630995424,
    -0.0011651675918590651121,
    -0.00021524167411495097282,
    0.00012805028238811618615,
    -0.000020134854780788238656,
    -1.2504934821426706573e-6,
    1.1330272319816958824e-6,
    -2.0563384169776071035e-7,
    6.1160951044814158179e-9,
    5.0020076444692229301e-9,
    -1.1812745704870201446e-9,
    1.0434267116911005105e-10,
    7.782263439905071254e-12,
    -3.6968056186422057082e-12,
    5.100370287454475979e-13,
    -2.0583260535665067832e-14,
    -5.3481225394230179824e-15,
    1.2267786282382607902e-15,
    -1.1812593016974587695e-16,
};

// Trapezoid buckets: upper x edge and step h (relative error <~ 3e-15 for
// nu up to 3.5, tuned against 30-digit references).
const double kTrapEdge[kTrapBuckets] = {3.0, 4.0, 8.0, 16.0, 32.0, 64.0, 128.0, 256.0, 1e300};
const double kTrapH[kTrapBuckets] = {0.2, 0.21, 0.19, 0.15, 0.105, 0.075, 0.053, 0.037, 0.022};
const double kTrapLo[kTrapBuckets] = {2.0, 3.0, 4.0, 8.0, 16.0, 32.0, 64.0, 128.0, 256.0};

// digamma(x), x > 0: the recurrence psi(x) = psi(x + 1) - 1/x up to x >= 10,
// then the asymptotic series psi(x) ~ ln x - 1/(2x) - sum_k B_2k / (2k x^2k)
// (Abramowitz & Stegun 6.3.5 and 6.3.18), seven terms: error below 1e-16.
double digamma(double x) {
  double acc = 0.0;
  while (x < 10.0) {
    acc -= 1.0 / x;
    x += 1.0;
  }
  const double r = 1.0 / (x * x);
  const double s = r * (1.0 / 12 - r * (1.0 / 120 - r * (1.0 / 252 - r * (1.0 / 240 - r * (1.0 / 132 -
                   r * (691.0 / 32760 - r * (1.0 / 12)))))));
  return acc + std::log(x) - 0.5 / x - s;
}
}  // namespace

bool matern_setup(double sigma2, double beta, double nu, MaternParams* p, double* tab) {
  if (!(std::isfinite(sigma2) && std::isfinite(beta) && std::isfinite(nu))) return false;
  if (!(beta > 0.0) || !(nu > 0.0) || sigma2 == 0.0) return false;
  *p = MaternParams{};
  p->sigma2 = sigma2;
  p->beta = beta;
  p->inv_beta = 1.0 / beta;
  p->nu = nu;
  p->norm = sigma2 / (std::pow(2.0, nu - 1.0) * std::tgamma(nu));
  if (nu == 0.5) p->kind = kNuHalf;
  else if (nu == 1.5) p->kind = kNuThreeHalves;
  else if (nu == 2.5) p->kind = kNuFiveHalves;
  else p->kind = kNuGeneral;
  for (int i = 0; i < kTabSize; ++i) tab[i] = 0.0;
  p->dparam = kDerivBeta;
  p->psi = digamma(nu);
  for (int k = 0; k < kDnuNodes; ++k) {   // nodes of dnu_ratio (every nu)
    const double t = k * kDnuH;
    const double sh = std::sinh(0.5 * t);
    tab[kTabDnu + k] = 2.0 * sh * sh;   // cosh t - 1 without cancellation
    tab[kTabDnu + kDnuNodes + k] = std::cosh(nu * t);
    tab[kTabDnu + 2 * kDnuNodes + k] = t * std::sinh(nu * t);
  }
  if (p->kind != kNuGeneral) return true;

  double mu;
  if (nu <= 0.5) {
    mu = -nu;
    p->pair_swapped = 1;
    p->nrec = 0;
  } else {
    const double N = std::floor(nu + 0.5);
    mu = nu - N;
    p->pair_swapped = 0;
    p->nrec = (int)N - 1;
  }
  p->mu = mu;
  // Gamma_1(mu) = (1/Gamma(1-mu) - 1/Gamma(1+mu)) / (2 mu) = -sum_odd a_k mu^(k-1)
  // Gamma_2(mu) = (1/Gamma(1-mu) + 1/Gamma(1+mu)) / 2     =  sum_even a_k mu^k
  double g1 = 0.0, g2 = 0.0;
  for (int k = 25; k >= 1; k -= 2) g1 = g1 * mu * mu + kRGamma[k];
  for (int k = 24; k >= 0; k -= 2) g2 = g2 * mu * mu + kRGamma[k];
  g1 = -g1;
  p->G1 = g1;
  p->G2 = g2;
  p->rgp = g2 - mu * g1;
  p->rgm = g2 + mu * g1;
  p->fac = (mu == 0.0) ? 1.0 : (M_PI * mu) / std::sin(M_PI * mu);
  double* t = tab + kTabTemme;
  for (int k = 1; k <= kTemmeTerms; ++k) {
    const double kd = (double)k;
    t[k - 1] = 1.0 / (kd - mu);
    t[kTemmeTerms + k - 1] = 1.0 / (kd + mu);
    t[2 * kTemmeTerms + k - 1] = 1.0 / (kd * kd - mu * mu);
    t[3 * kTemmeTerms + k - 1] = 1.0 / kd;
  }
  for (int b = 0; b < kTrapBuckets; ++b) {
    const double h = kTrapH[b];
    p->trap_h[b] = h;
    double* base = tab + kTabTrap + b * 3 * kTrapTerms;
    int n = 0;
    for (int k = 0; k < kTrapTerms; ++k) {
      const double tk = (k + 1) * h;
      const double cm1 = std::cosh(tk) - 1.0;
      base[k] = cm1;
      base[kTrapTerms + k] = std::cosh(nu * tk);
      base[2 * kTrapTerms + k] = std::cosh((nu - 1.0) * tk);
      n = k + 1;
      if (kTrapLo[b] * cm1 > 42.0) break;
    }
    p->trap_n[b] = n;
  }
  (void)kTrapEdge;
  return true;
}

// Writes out[b * ld + a] = C(||s_{r0+a} - s_{c0+b}||) (or dC/dbeta) for a < m, b < ncol.
template <bool deriv>
__global__ void __launch_bounds__(256) matern_block_kernel(MaternParams p, const double* __restrict__ x,
                                                           const double* __restrict__ y, int64_t r0, int64_t m,
                                                           int64_t c0, int64_t ncol, double* __restrict__ out,
                                                           int64_t ld) {
  const int64_t a = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t b = blockIdx.y;
  if (a >= m || b >= ncol) return;
  const double r = loc_dist(p, x, y, r0 + a, c0 + b);
  double c, dc;
  matern_eval<deriv>(p, r, c, dc);
  out[b * ld + a] = deriv ? dc : c;
}

hipError_t launch_matern_block(const MaternParams& p, const double* x, const double* y, int64_t r0, int64_t m,
                               int64_t c0, int64_t ncol, double* out, int64_t ld, bool deriv, hipStream_t s) {
  if (m <= 0 || ncol <= 0) return hipSuccess;
  for (int64_t cb = 0; cb < ncol; cb += 65535) {
    const int64_t nc = (ncol - cb < 65535) ? ncol - cb : 65535;
    dim3 grid((unsigned)((m + 255) / 256), (unsigned)nc);
    if (deriv)
      hipLaunchKernelGGL(matern_block_kernel<true>, grid, dim3(256), 0, s, p, x, y, r0, m, c0 + cb, nc,
                         out + cb * ld, ld);
    else
      hipLaunchKernelGGL(matern_block_kernel<false>, grid, dim3(256), 0, s, p, x, y, r0, m, c0 + cb, nc,
                         out + cb * ld, ld);
  }
  return hipGetLastError();
}

}  // namespace tlrk
