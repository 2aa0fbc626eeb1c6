"""Exact (dense) log-likelihood and score with Sigma held as its lower tiles.

TEST INFRASTRUCTURE ONLY (see the package docstring): nothing in the product
imports or runs this module.

The quantities are the plain definitions of ``dense.py``:
  * Eq. (1) (Section III): l = -n/2 log(2 pi) - 1/2 log|Sigma| - 1/2 z^T Sigma^{-1} z,
    log|Sigma| = 2 sum log diag(L), z^T Sigma^{-1} z = ||L^{-1} z||^2;
  * the score dl/dtheta_i = -1/2 tr(Sigma^{-1} dSigma_i) + 1/2 a^T dSigma_i a,
    a = Sigma^{-1} z (not in the paper, which optimises without derivatives);
  * the measurement generator z = L eps (Section VIII-D).
Only the storage differs: Sigma is never formed as one n x n array (a full
40,000^2 matrix breaks the host LAPACK Cholesky, and 102,400^2 does not fit in
host memory).  The lower tiles A_ij (i >= j) of size nb are generated from
Eq. (MaternCov) one by one and factored by the textbook right-looking blocked
Cholesky, each step a LAPACK/BLAS call on whole tiles:
    for k = 0 .. NT-1:
        L_kk = chol(A_kk)                       (dpotrf)
        L_ik = A_ik L_kk^{-T}        i > k      (dtrsm)
        A_ij -= L_ik L_jk^T          i >= j > k (dgemm)
For the score, Sigma^{-1} is formed in the same storage: M = L^{-1} from
L M = I block by block (M_jj = L_jj^{-1}, M_ij = -L_ii^{-1} sum_{j<=k<i} L_ik M_kj),
then the lower tiles of Sigma^{-1} = M^T M, S_ij = sum_{k>=i} M_ki^T M_kj.
The tile size changes only the rounding order, never the result.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.linalg import blas, lapack

from . import matern as _m
from .dense import NotSPDError


def _bounds(n: int, nb: int) -> list[tuple[int, int]]:
    nt = (n + nb - 1) // nb
    return [(t * nb, min(n, (t + 1) * nb)) for t in range(nt)]


class LowerTiles:
    """Lower tiles T[i][j] (i >= j, Fortran order) of an n x n symmetric matrix."""

    def __init__(self, n: int, nb: int):
        if n < 1 or nb < 1:
            raise ValueError("n and nb must be >= 1")
        self.n, self.nb = int(n), int(nb)
        self.b = _bounds(self.n, self.nb)
        self.nt = len(self.b)
        self.t = [[None] * (i + 1) for i in range(self.nt)]

    def sl(self, i: int) -> slice:
        return slice(*self.b[i])

    def to_dense(self) -> np.ndarray:
        """Full symmetric matrix (lower tiles mirrored); small n only."""
        A = np.zeros((self.n, self.n))
        for i in range(self.nt):
            for j in range(i + 1):
                A[self.sl(i), self.sl(j)] = self.t[i][j]
                if i != j:
                    A[self.sl(j), self.sl(i)] = self.t[i][j].T
        return A


def covariance_tiles(x, y, theta, nb: int, deriv: bool = False) -> LowerTiles:
    """Lower tiles of Sigma(theta) (Eq. (MaternCov)) or of dSigma/dbeta."""
    x = np.asarray(x, float)
    y = np.asarray(y, float)
    T = LowerTiles(x.shape[0], nb)
    f = _m.covariance_dbeta if deriv else _m.covariance
    for i in range(T.nt):
        for j in range(i + 1):
            T.t[i][j] = np.asfortranarray(f(x, y, theta, rows=T.sl(i), cols=T.sl(j)))
    return T


def cholesky_tiles(A: LowerTiles) -> LowerTiles:
    """Right-looking blocked Cholesky in place: A's tiles become L's.

    The diagonal tiles come back lower triangular (zeros above).  A
    non-positive pivot raises NotSPDError with its 1-based global row.
    """
    for k in range(A.nt):
        c, info = lapack.dpotrf(A.t[k][k], lower=1, clean=1, overwrite_a=1)
        if info > 0:
            raise NotSPDError(A.b[k][0] + info)
        if info < 0:
            raise ValueError(f"dpotrf argument {-info} invalid")
        A.t[k][k] = c
        for i in range(k + 1, A.nt):
            # L_ik = A_ik L_kk^{-T}: solve X L_kk^T = A_ik from the right
            A.t[i][k] = blas.dtrsm(1.0, c, A.t[i][k], side=1, lower=1, trans_a=1, overwrite_b=1)
        for j in range(k + 1, A.nt):
            for i in range(j, A.nt):
                A.t[i][j] = blas.dgemm(-1.0, A.t[i][k], A.t[j][k], beta=1.0, c=A.t[i][j],
                                       trans_b=1, overwrite_c=1)
    return A


def forward_solve(L: LowerTiles, z) -> np.ndarray:
    """y = L^{-1} z: y_k = L_kk^{-1} (z_k - sum_{j<k} L_kj y_j)."""
    y = np.array(z, dtype=np.float64, copy=True)
    for k in range(L.nt):
        r = y[L.sl(k)]
        for j in range(k):
            r -= L.t[k][j] @ y[L.sl(j)]
        y[L.sl(k)] = blas.dtrsv(L.t[k][k], r, lower=1)
    return y


def backward_solve(L: LowerTiles, w) -> np.ndarray:
    """a = L^{-T} w: a_k = L_kk^{-T} (w_k - sum_{i>k} L_ik^T a_i), k descending."""
    a = np.array(w, dtype=np.float64, copy=True)
    for k in range(L.nt - 1, -1, -1):
        r = a[L.sl(k)]
        for i in range(k + 1, L.nt):
            r -= L.t[i][k].T @ a[L.sl(i)]
        a[L.sl(k)] = blas.dtrsv(L.t[k][k], r, lower=1, trans=1)
    return a


def lower_matvec(L: LowerTiles, v) -> np.ndarray:
    """L v for a lower-triangular L held in tiles."""
    v = np.asarray(v, dtype=np.float64)
    out = np.zeros(L.n)
    for i in range(L.nt):
        for j in range(i + 1):
            out[L.sl(i)] += L.t[i][j] @ v[L.sl(j)]
    return out


def inverse_tiles(L: LowerTiles) -> LowerTiles:
    """Lower tiles of Sigma^{-1} = L^{-T} L^{-1} from the Cholesky tiles.

    M = L^{-1} column by column from L M = I, then S = M^T M.  L is left
    unchanged; the result needs a second tile set.
    """
    M = LowerTiles(L.n, L.nb)
    eye = [np.eye(L.b[k][1] - L.b[k][0], order="F") for k in range(L.nt)]
    for j in range(L.nt):
        M.t[j][j] = blas.dtrsm(1.0, L.t[j][j], eye[j], lower=1)
        for i in range(j + 1, L.nt):
            acc = np.zeros((L.b[i][1] - L.b[i][0], L.b[j][1] - L.b[j][0]), order="F")
            for k in range(j, i):
                acc = blas.dgemm(1.0, L.t[i][k], M.t[k][j], beta=1.0, c=acc, overwrite_c=1)
            M.t[i][j] = blas.dtrsm(-1.0, L.t[i][i], acc, lower=1, overwrite_b=1)
    # S_ij = sum_{k >= i} M_ki^T M_kj, in place: rows top to bottom, S_ii last in its row
    for i in range(L.nt):
        for j in range(i + 1):
            acc = np.zeros((L.b[i][1] - L.b[i][0], L.b[j][1] - L.b[j][0]), order="F")
            for k in range(i, L.nt):
                acc = blas.dgemm(1.0, M.t[k][i], M.t[k][j], beta=1.0, c=acc, trans_a=1, overwrite_c=1)
            M.t[i][j] = acc
    return M


def _ll(n: int, logdet: float, quad: float) -> float:
    return -0.5 * n * math.log(2.0 * math.pi) - 0.5 * logdet - 0.5 * quad


def loglik(x, y, z, theta, nb: int = 2000) -> dict:
    """Eq. (1) with a tiled Cholesky: {'ll', 'logdet', 'quad', 'n'}."""
    L = cholesky_tiles(covariance_tiles(x, y, theta, nb))
    logdet = 2.0 * sum(float(np.sum(np.log(np.diag(L.t[k][k])))) for k in range(L.nt))
    w = forward_solve(L, z)
    quad = float(w @ w)
    return {"ll": _ll(L.n, logdet, quad), "logdet": logdet, "quad": quad, "n": L.n}


def gradient(x, y, z, theta, nb: int = 2000) -> dict:
    """Score in (sigma^2, beta), as ``dense.gradient``, with tiled storage.

    Returns {'ll', 'logdet', 'quad', 'dsigma2', 'dbeta', 'tr_beta', 'qf_beta'}.
    The sigma^2 terms use dSigma/dsigma^2 = Sigma(1, beta, nu) tile by tile;
    both dSigma tiles are generated where they are contracted.
    """
    sigma2, beta, nu = (float(t) for t in theta)
    L = cholesky_tiles(covariance_tiles(x, y, theta, nb))
    logdet = 2.0 * sum(float(np.sum(np.log(np.diag(L.t[k][k])))) for k in range(L.nt))
    w = forward_solve(L, z)
    quad = float(w @ w)
    alpha = backward_solve(L, w)
    S = inverse_tiles(L)
    del L
    x = np.asarray(x, float)
    y = np.asarray(y, float)
    tr_s2 = tr_b = qf_s2 = qf_b = 0.0
    for i in range(S.nt):
        for j in range(i + 1):
            wgt = 1.0 if i == j else 2.0  # the upper tile (j, i) is the transpose
            dS2 = _m.covariance(x, y, (1.0, beta, nu), rows=S.sl(i), cols=S.sl(j))
            dB = _m.covariance_dbeta(x, y, theta, rows=S.sl(i), cols=S.sl(j))
            ai, aj = alpha[S.sl(i)], alpha[S.sl(j)]
            tr_s2 += wgt * float(np.sum(S.t[i][j] * dS2))
            tr_b += wgt * float(np.sum(S.t[i][j] * dB))
            qf_s2 += wgt * float(ai @ (dS2 @ aj))
            qf_b += wgt * float(ai @ (dB @ aj))
    return {"ll": _ll(S.n, logdet, quad), "logdet": logdet, "quad": quad,
            "dsigma2": -0.5 * tr_s2 + 0.5 * qf_s2,
            "dbeta": -0.5 * tr_b + 0.5 * qf_b,
            "tr_beta": tr_b, "qf_beta": qf_b}


def sample_z(x, y, theta, eps, nb: int = 2000) -> np.ndarray:
    """z = L eps with L the Cholesky factor of Sigma(theta) (Section VIII-D)."""
    L = cholesky_tiles(covariance_tiles(x, y, theta, nb))
    return lower_matvec(L, eps)
