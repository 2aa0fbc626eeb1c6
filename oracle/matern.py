"""Matérn covariance (paper Section IV, Eq. (MaternCov)) in FP64.

C(r; theta) = theta1 / (2^(theta3 - 1) Gamma(theta3)) * (r/theta2)^theta3
              * K_theta3(r / theta2)
with theta = (variance sigma^2, range beta, smoothness nu).  K is the modified
Bessel function of the second kind (scipy.special.kv here).

At r = 0 the formula is 0 * infinity; the limit u^nu K_nu(u) -> 2^(nu-1)
Gamma(nu) gives C(0) = theta1, used whenever r == 0 exactly.
"""
from __future__ import annotations

import numpy as np
from scipy.special import digamma, gamma, kv


def matern(r, sigma2: float, beta: float, nu: float) -> np.ndarray:
    """C(r; sigma2, beta, nu), Eq. (MaternCov); C(0) = sigma2."""
    r = np.asarray(r, dtype=np.float64)
    u = r / beta
    out = np.full(u.shape, float(sigma2))
    pos = u > 0
    up = u[pos]
    out[pos] = sigma2 / (2.0 ** (nu - 1.0) * gamma(nu)) * up ** nu * kv(nu, up)
    return out


def dmatern_dbeta(r, sigma2: float, beta: float, nu: float) -> np.ndarray:
    """dC/dbeta of Eq. (MaternCov).

    With u = r/beta, d/du [u^nu K_nu(u)] = -u^nu K_{nu-1}(u) (standard Bessel
    identity) and du/dbeta = -u/beta, so
    dC/dbeta = sigma2 / (2^(nu-1) Gamma(nu)) * u^(nu+1) K_{nu-1}(u) / beta,
    which is 0 at r = 0.  K_{-mu} = K_mu covers nu < 1.
    """
    r = np.asarray(r, dtype=np.float64)
    u = r / beta
    out = np.zeros(u.shape)
    pos = u > 0
    up = u[pos]
    out[pos] = (sigma2 / (2.0 ** (nu - 1.0) * gamma(nu)) * up ** (nu + 1.0)
                * kv(nu - 1.0, up) / beta)
    return out


def dkv_dnu(nu: float, x) -> np.ndarray:
    """dK_nu(x)/dnu, the derivative of scipy's K_nu in its order.

    Central differences D(h) = (K_{nu+h} - K_{nu-h}) / (2h) at h and h/2,
    combined by Richardson extrapolation, (4 D(h/2) - D(h)) / 3, whose error is
    O(h^4) (h = 2e-3; scipy's K_nu itself is accurate to about 1e-14
    relative, so the result to about 1e-10).
    """
    x = np.asarray(x, dtype=np.float64)
    h = 2e-3

    def d(hh):
        return (kv(nu + hh, x) - kv(nu - hh, x)) / (2.0 * hh)
    return (4.0 * d(h / 2.0) - d(h)) / 3.0


def dmatern_dnu(r, sigma2: float, beta: float, nu: float) -> np.ndarray:
    """dC/dnu of Eq. (MaternCov): with u = r / beta,
    dC/dnu = C (log(u / 2) - psi(nu)) + sigma2 2^{1-nu} / Gamma(nu) u^nu dK_nu/dnu(u)
    (psi the digamma function); 0 at r = 0, where C = sigma2 for every nu."""
    r = np.asarray(r, dtype=np.float64)
    u = r / beta
    out = np.zeros(u.shape)
    pos = u > 0
    up = u[pos]
    norm = sigma2 / (2.0 ** (nu - 1.0) * gamma(nu))
    c = norm * up ** nu * kv(nu, up)
    out[pos] = c * (np.log(up / 2.0) - digamma(nu)) + norm * up ** nu * dkv_dnu(nu, up)
    return out


EARTH_RADIUS_KM = 6371.0


def distances(xa, ya, xb, yb, metric: str = "euclid", radius: float = EARTH_RADIUS_KM) -> np.ndarray:
    """Distance matrix r[a, b] between locations (Section IV).

    "euclid": ||s_a - s_b||_2.  "great_circle": Eq. (gcd), the haversine
    formula, with x the longitude and y the latitude in degrees:
    hav(d / r) = hav(phi_b - phi_a) + cos(phi_a) cos(phi_b) hav(lam_b - lam_a),
    hav(t) = sin^2(t / 2), solved for d = 2 r arcsin(sqrt(hav(d / r))).
    """
    xa, ya, xb, yb = (np.asarray(v, float) for v in (xa, ya, xb, yb))
    if metric == "euclid":
        dx = np.subtract.outer(xa, xb)
        dy = np.subtract.outer(ya, yb)
        return np.sqrt(dx * dx + dy * dy)
    if metric != "great_circle":
        raise ValueError(metric)
    phi_a, phi_b = np.radians(ya), np.radians(yb)
    lam_a, lam_b = np.radians(xa), np.radians(xb)

    def hav(t):
        return np.sin(t / 2.0) ** 2

    h = hav(np.subtract.outer(phi_b, phi_a).T) + np.outer(np.cos(phi_a), np.cos(phi_b)) * hav(
        np.subtract.outer(lam_b, lam_a).T)
    return 2.0 * radius * np.arcsin(np.sqrt(np.clip(h, 0.0, 1.0)))


def covariance(x, y, theta, rows=None, cols=None, metric: str = "euclid",
               radius: float = EARTH_RADIUS_KM) -> np.ndarray:
    """Sigma(theta)[rows, cols] with Sigma_ab = C(d(s_a, s_b); theta) (Section III)."""
    x = np.asarray(x, float)
    y = np.asarray(y, float)
    ra = slice(None) if rows is None else rows
    cb = slice(None) if cols is None else cols
    return matern(distances(x[ra], y[ra], x[cb], y[cb], metric, radius), *theta)


def covariance_dbeta(x, y, theta, rows=None, cols=None, metric: str = "euclid",
                     radius: float = EARTH_RADIUS_KM) -> np.ndarray:
    """dSigma/dbeta[rows, cols], entry-wise dC/dbeta."""
    x = np.asarray(x, float)
    y = np.asarray(y, float)
    ra = slice(None) if rows is None else rows
    cb = slice(None) if cols is None else cols
    return dmatern_dbeta(distances(x[ra], y[ra], x[cb], y[cb], metric, radius), *theta)


def covariance_dnu(x, y, theta, rows=None, cols=None, metric: str = "euclid",
                   radius: float = EARTH_RADIUS_KM) -> np.ndarray:
    """dSigma/dnu[rows, cols], entry-wise dC/dnu."""
    x = np.asarray(x, float)
    y = np.asarray(y, float)
    ra = slice(None) if rows is None else rows
    cb = slice(None) if cols is None else cols
    return dmatern_dnu(distances(x[ra], y[ra], x[cb], y[cb], metric, radius), *theta)


def cross_covariance(xa, ya, xb, yb, theta, metric: str = "euclid", radius: float = EARTH_RADIUS_KM):
    """C(d(a_i, b_j); theta) between two location sets (Sigma_12 of Section III)."""
    return matern(distances(xa, ya, xb, yb, metric, radius), *theta)
