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
from scipy.special import gamma, kv


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


def distances(xa, ya, xb, yb) -> np.ndarray:
    """Euclidean distance matrix r[a, b] = ||s_a - s_b|| (Section IV)."""
    dx = np.subtract.outer(np.asarray(xa, float), np.asarray(xb, float))
    dy = np.subtract.outer(np.asarray(ya, float), np.asarray(yb, float))
    return np.sqrt(dx * dx + dy * dy)


def covariance(x, y, theta, rows=None, cols=None) -> np.ndarray:
    """Sigma(theta)[rows, cols] with Sigma_ab = C(||s_a - s_b||; theta) (Section III)."""
    x = np.asarray(x, float)
    y = np.asarray(y, float)
    ra = slice(None) if rows is None else rows
    cb = slice(None) if cols is None else cols
    return matern(distances(x[ra], y[ra], x[cb], y[cb]), *theta)


def covariance_dbeta(x, y, theta, rows=None, cols=None) -> np.ndarray:
    """dSigma/dbeta[rows, cols], entry-wise dC/dbeta."""
    x = np.asarray(x, float)
    y = np.asarray(y, float)
    ra = slice(None) if rows is None else rows
    cb = slice(None) if cols is None else cols
    return dmatern_dbeta(distances(x[ra], y[ra], x[cb], y[cb]), *theta)
