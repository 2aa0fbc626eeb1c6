"""Kriging prediction (Section III), FP64, plain definitions.

TEST INFRASTRUCTURE ONLY (see the package docstring).

With [Z_1; Z_2] jointly Gaussian, zero mean, covariance blocks Sigma_11
(m x m), Sigma_12 (m x n), Sigma_22 (n x n) from Eq. (MaternCov):
  * Eq. (pred3): the prediction Z_1 = Sigma_12 Sigma_22^{-1} Z_2;
  * Eq. (pred2): the conditional covariance Sigma_11 - Sigma_12 Sigma_22^{-1} Sigma_21,
    whose diagonal is the prediction variance;
  * the mean squared error of a prediction against the true values (the
    paper's accuracy measure for prediction, Section VIII-D):
    MSE = (1/m) sum_i (Z_1,i - Z_1,i^true)^2.
Sigma_22^{-1} is applied through its Cholesky factor (LAPACK), as the paper
describes the prediction step.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import solve_triangular

from . import matern as _m
from .dense import cholesky_lower


def predict(x, y, z, xnew, ynew, theta, metric: str = "euclid", variance: bool = False):
    """Eq. (pred3) (and the diagonal of Eq. (pred2) if variance)."""
    S22 = _m.covariance(x, y, theta, metric=metric)
    S12 = _m.cross_covariance(xnew, ynew, x, y, theta, metric=metric)
    L = cholesky_lower(S22)
    a = solve_triangular(L, solve_triangular(L, np.asarray(z, float), lower=True), lower=True, trans="T")
    pred = S12 @ a
    if not variance:
        return pred
    W = solve_triangular(L, S12.T, lower=True)
    var = float(theta[0]) - np.sum(W * W, axis=0)
    return pred, var


def mse(pred, truth) -> float:
    """Mean squared prediction error."""
    d = np.asarray(pred, float) - np.asarray(truth, float)
    return float(np.mean(d * d))
