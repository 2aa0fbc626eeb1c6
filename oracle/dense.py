"""Exact (dense) Gaussian log-likelihood and its gradient, FP64.

Plain definitions, written out:

* Eq. (1) (Section III):
      l(theta) = -n/2 log(2 pi) - 1/2 log|Sigma(theta)| - 1/2 z^T Sigma^{-1} z
  with Sigma = L L^T (LAPACK dpotrf, lower), log|Sigma| = 2 sum_i log L_ii and
  z^T Sigma^{-1} z = ||L^{-1} z||^2 (the Cholesky, log-determinant and solve
  named in Section III and in the task list of Section VI).  Logarithms are
  natural.
* Gradient (not in the paper, whose optimiser is derivative-free): the
  textbook score
      dl/dtheta_i = -1/2 tr(Sigma^{-1} dSigma/dtheta_i)
                    + 1/2 alpha^T (dSigma/dtheta_i) alpha,  alpha = Sigma^{-1} z,
  with dSigma/dsigma2 = Sigma(1, beta, nu) and dSigma/dbeta entry-wise from
  ``matern.dmatern_dbeta``; Sigma^{-1} is formed explicitly from the factor.
* Measurements (Section VIII-D, "exact computation" of synthetic data):
  z = L eps with L the dense Cholesky factor of Sigma(theta_true).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.linalg import lapack, solve_triangular

from . import matern as _m


class NotSPDError(ArithmeticError):
    """Cholesky met a non-positive pivot; ``info`` is its 1-based global row."""

    def __init__(self, info: int):
        super().__init__(f"matrix not positive definite at row {info}")
        self.info = int(info)


def cholesky_lower(S: np.ndarray) -> np.ndarray:
    """Lower Cholesky factor by LAPACK dpotrf; NotSPDError(info) on failure."""
    c, info = lapack.dpotrf(np.asfortranarray(S), lower=1, clean=1, overwrite_a=0)
    if info > 0:
        raise NotSPDError(info)
    if info < 0:
        raise ValueError(f"dpotrf argument {-info} invalid")
    return c


def loglik(x, y, z, theta) -> dict:
    """Eq. (1): returns {'ll', 'logdet', 'quad', 'n'}."""
    z = np.asarray(z, dtype=np.float64)
    n = z.shape[0]
    S = _m.covariance(x, y, theta)
    L = cholesky_lower(S)
    logdet = 2.0 * float(np.sum(np.log(np.diag(L))))
    w = solve_triangular(L, z, lower=True)
    quad = float(w @ w)
    ll = -0.5 * n * math.log(2.0 * math.pi) - 0.5 * logdet - 0.5 * quad
    return {"ll": ll, "logdet": logdet, "quad": quad, "n": n}


def gradient(x, y, z, theta) -> dict:
    """Score in (sigma2, beta, nu) by the textbook formula; also returns l.

    Returns {'ll', 'logdet', 'quad', 'dsigma2', 'dbeta', 'dnu', 'tr_beta',
    'qf_beta', 'tr_nu', 'qf_nu'} where tr_beta = tr(Sigma^{-1} dSigma/dbeta)
    and qf_beta = alpha^T dSigma/dbeta alpha (likewise for nu).
    """
    sigma2, beta, nu = (float(t) for t in theta)
    z = np.asarray(z, dtype=np.float64)
    n = z.shape[0]
    S = _m.covariance(x, y, theta)
    L = cholesky_lower(S)
    logdet = 2.0 * float(np.sum(np.log(np.diag(L))))
    w = solve_triangular(L, z, lower=True)
    quad = float(w @ w)
    ll = -0.5 * n * math.log(2.0 * math.pi) - 0.5 * logdet - 0.5 * quad
    Linv = solve_triangular(L, np.eye(n), lower=True)
    Sinv = Linv.T @ Linv
    alpha = Sinv @ z
    dS_s2 = _m.covariance(x, y, (1.0, beta, nu))
    dS_b = _m.covariance_dbeta(x, y, theta)
    dS_n = _m.covariance_dnu(x, y, theta)
    tr_s2 = float(np.sum(Sinv * dS_s2))
    tr_b = float(np.sum(Sinv * dS_b))
    tr_n = float(np.sum(Sinv * dS_n))
    qf_s2 = float(alpha @ (dS_s2 @ alpha))
    qf_b = float(alpha @ (dS_b @ alpha))
    qf_n = float(alpha @ (dS_n @ alpha))
    return {"ll": ll, "logdet": logdet, "quad": quad,
            "dsigma2": -0.5 * tr_s2 + 0.5 * qf_s2,
            "dbeta": -0.5 * tr_b + 0.5 * qf_b,
            "dnu": -0.5 * tr_n + 0.5 * qf_n,
            "tr_beta": tr_b, "qf_beta": qf_b, "tr_nu": tr_n, "qf_nu": qf_n}


def sample_z(x, y, theta, eps) -> np.ndarray:
    """z = L eps with L = chol(Sigma(theta)) (Section VIII-D)."""
    L = cholesky_lower(_m.covariance(x, y, theta))
    return L @ np.asarray(eps, dtype=np.float64)
