// Device evaluation of the Matérn covariance (Section IV, Eq. (MaternCov)) and
// of its derivative in the range parameter beta.
//
// K_nu is evaluated from published mathematics, not from any library source:
//  * x <= 2: Temme's series (N. M. Temme, J. Comput. Phys. 19 (1975) 324-337)
//    for K_mu and K_{mu+1}, |mu| <= 1/2, followed by the forward recurrence
//    K_{v+1} = K_{v-1} + (2 v / x) K_v (DLMF 10.29.1);
//  * x > 2: the integral K_v(x) = int_0^inf exp(-x cosh t) cosh(v t) dt
//    (DLMF 10.32.9) by the trapezoidal rule, whose error decays geometrically
//    for this analytic integrand (Trefethen & Weideman, SIAM Rev. 56 (2014));
//    the step is chosen per x-bucket so the relative error stays ~1e-15;
//  * nu = 1/2, 3/2, 5/2: the elementary closed forms of K_{n+1/2}.
// exp/log/sqrt are HIP's device functions.
#pragma once
#include "common.h"

namespace tlrk {

// Returns (a, b) = (K_mu(x), K_{mu+1}(x)) by Temme's series, x in (0, 2].
__device__ inline void temme_pair(const MaternParams& p, double x, double& ka, double& kb) {
  const double* inv_kmm = p.tab + kTabTemme;
  const double* inv_kpm = inv_kmm + kTemmeTerms;
  const double* inv_k2 = inv_kpm + kTemmeTerms;
  const double* inv_k = inv_k2 + kTemmeTerms;
  const double mu = p.mu;
  const double lx = log(2.0 / x);            // ln(2/x)
  const double sig = mu * lx;
  const double e = exp(sig);                 // (2/x)^mu
  const double ch = 0.5 * (e + 1.0 / e);
  const double shs = (fabs(sig) < 1e-8) ? (1.0 + sig * sig * (1.0 / 6.0)) : 0.5 * (e - 1.0 / e) / sig;
  double f = p.fac * (ch * p.G1 + shs * lx * p.G2);
  double pk = 0.5 * e / p.rgp;               // (x/2)^-mu Gamma(1+mu) / 2
  double qk = 0.5 / (e * p.rgm);             // (x/2)^mu Gamma(1-mu) / 2
  const double x2 = 0.25 * x * x;
  double c = 1.0;
  double s0 = f, s1 = pk;
  for (int k = 1; k <= kTemmeTerms; ++k) {
    const double kd = (double)k;
    f = (kd * f + pk + qk) * inv_k2[k - 1];
    pk *= inv_kmm[k - 1];
    qk *= inv_kpm[k - 1];
    c *= x2 * inv_k[k - 1];
    const double d0 = c * f;
    const double d1 = c * (pk - kd * f);
    s0 += d0;
    s1 += d1;
    if (fabs(d0) < 1e-17 * fabs(s0) && fabs(d1) < 1e-17 * fabs(s1)) break;
  }
  ka = s0;
  kb = 2.0 / x * s1;
}

// Returns e^x K_nu(x) and e^x K_{nu-1}(x) by the trapezoidal rule, x > 2.
__device__ inline void trap_pair(const MaternParams& p, double x, double& knu, double& knum1) {
  int b;
  if (x <= 3.0) b = 0;
  else if (x <= 4.0) b = 1;
  else if (x <= 8.0) b = 2;
  else if (x <= 16.0) b = 3;
  else if (x <= 32.0) b = 4;
  else if (x <= 64.0) b = 5;
  else if (x <= 128.0) b = 6;
  else if (x <= 256.0) b = 7;
  else b = 8;
  const double* base = p.tab + kTabTrap + b * 3 * kTrapTerms;
  const double* cm1 = base;
  const double* wnu = base + kTrapTerms;
  const double* wnm = base + 2 * kTrapTerms;
  double s = 0.5, sm = 0.5;
  const int nt = p.trap_n[b];
  for (int k = 0; k < nt; ++k) {
    const double a = x * cm1[k];
    if (a > 42.0) break;
    const double g = exp(-a);
    s += g * wnu[k];
    sm += g * wnm[k];
  }
  knu = p.trap_h[b] * s;
  knum1 = p.trap_h[b] * sm;
}

// S1 / S0 with S0 = sum_k w_k e^{-x (cosh t_k - 1)} cosh(nu t_k) and
// S1 = sum_k e^{-x (cosh t_k - 1)} t_k sinh(nu t_k), t_k = k h, w_0 = 1/2:
// the trapezoid rule on K_nu(x) = int_0^inf e^{-x cosh t} cosh(nu t) dt
// (DLMF 10.32.9) and on its derivative in the order,
// dK_nu/dnu(x) = int_0^inf e^{-x cosh t} t sinh(nu t) dt, with the common
// factor e^{-x} dropped, so S1 / S0 = (dK_nu/dnu) / K_nu.  Both integrands
// are even and analytic in the strip |Im t| < pi/2, so the trapezoid error
// falls like exp(-pi^2 / h) (Trefethen & Weideman); the sum stops once
// x (cosh t_k - 1) exceeds nu t_k + 40 (past the peak, terms below e^-40).
__device__ inline double dnu_ratio(const MaternParams& p, double x) {
  const double* cm1 = p.tab + kTabDnu;
  const double* cnu = cm1 + kDnuNodes;
  const double* tsn = cnu + kDnuNodes;
  double s0 = 0.5, s1 = 0.0;
  for (int k = 1; k < kDnuNodes; ++k) {
    const double a = x * cm1[k];
    if (a > 40.0 + p.nu * (k * kDnuH)) break;
    const double e = exp(-a);
    s0 += e * cnu[k];
    s1 += e * tsn[k];
  }
  return s1 / s0;
}

// Matérn value C(r) and, if want_d, its derivative in the parameter p.dparam
// selects: dC/dbeta, or
//   dC/dnu = C (log(u / 2) - psi(nu)) + sigma2 2^{1-nu} / Gamma(nu) u^nu dK_nu/dnu(u)
//          = C (log(u / 2) - psi(nu) + (dK_nu/dnu)(u) / K_nu(u)),
// which is 0 at r = 0 (C(0) = sigma2 for every nu) and is taken as 0 below
// u = 1e-10 (its limit; the trapezoid's nodes end there).
template <bool want_d>
__device__ inline void matern_eval(const MaternParams& p, double r, double& c, double& dc) {
  if (r == 0.0) {  // limit u^nu K_nu(u) -> 2^(nu-1) Gamma(nu)
    c = p.sigma2;
    dc = 0.0;
    return;
  }
  if (want_d && p.dparam == kDerivNu) {
    double unused;
    matern_eval<false>(p, r, c, unused);
    const double u = r * p.inv_beta;
    dc = (u < 1e-10) ? 0.0 : c * (log(0.5 * u) - p.psi + dnu_ratio(p, u));
    return;
  }
  const double u = r * p.inv_beta;
  if (p.kind == kNuHalf) {
    const double e = exp(-u);
    c = p.sigma2 * e;
    if (want_d) dc = p.sigma2 * u * e * p.inv_beta;
    return;
  }
  if (p.kind == kNuThreeHalves) {
    const double e = exp(-u);
    c = p.sigma2 * (1.0 + u) * e;
    if (want_d) dc = p.sigma2 * u * u * e * p.inv_beta;
    return;
  }
  if (p.kind == kNuFiveHalves) {
    const double e = exp(-u);
    c = p.sigma2 * (1.0 + u + u * u * (1.0 / 3.0)) * e;
    if (want_d) dc = p.sigma2 * (1.0 / 3.0) * u * u * (1.0 + u) * e * p.inv_beta;
    return;
  }
  // general nu: need K_nu(u) and K_{nu-1}(u)
  if (u > 700.0) { c = 0.0; dc = 0.0; return; }
  double knu, knm;
  double scale;  // multiplies u^nu * K
  if (u <= 2.0) {
    double ka, kb;
    temme_pair(p, u, ka, kb);
    if (p.pair_swapped) {
      knu = ka; knm = kb;   // (K_{-nu}, K_{1-nu}) = (K_nu, K_{nu-1})
    } else {
      // (K_mu, K_{mu+1}); step up nrec times to (K_{nu-1}, K_nu)
      double v = p.mu + 1.0;
      const double ix2 = 2.0 / u;
      for (int s = 0; s < p.nrec; ++s) {
        const double kn = ka + v * ix2 * kb;
        ka = kb; kb = kn; v += 1.0;
      }
      knm = ka; knu = kb;
    }
    scale = exp(p.nu * log(u));
  } else {
    trap_pair(p, u, knu, knm);
    scale = exp(p.nu * log(u) - u);
  }
  c = p.norm * scale * knu;
  if (want_d) dc = p.norm * scale * u * knm * p.inv_beta;
}

// Distance of two locations (Section IV).  Euclidean: sqrt(dx^2 + dy^2).
// Great circle, Eq. (gcd): with phi the latitudes (y) and lambda the
// longitudes (x) in radians, hav(d / r) = hav(phi_b - phi_a) +
// cos(phi_a) cos(phi_b) hav(lambda_b - lambda_a), hav(t) = sin^2(t / 2), so
// d = 2 r asin(sqrt(h)) (h clamped to 1 against rounding).
__device__ inline double point_dist(const MaternParams& p, double xa, double ya, double xb, double yb) {
  if (p.metric == kMetricGreatCircle) {
    constexpr double kDeg = 3.14159265358979323846 / 180.0;
    const double sp = sin(0.5 * kDeg * (yb - ya));
    const double sl = sin(0.5 * kDeg * (xb - xa));
    const double h = sp * sp + cos(kDeg * ya) * cos(kDeg * yb) * (sl * sl);
    return 2.0 * p.radius * asin(sqrt(h < 1.0 ? h : 1.0));
  }
  const double dx = xa - xb;
  const double dy = ya - yb;
  return sqrt(dx * dx + dy * dy);
}

__device__ inline double loc_dist(const MaternParams& p, const double* __restrict__ x,
                                  const double* __restrict__ y, int64_t a, int64_t b) {
  return point_dist(p, x[a], y[a], x[b], y[b]);
}

}  // namespace tlrk
