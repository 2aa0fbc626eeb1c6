"""CPU tile low-rank (TLR) log-likelihood, FP64 (paper Section V).

The paper compresses each off-diagonal tile of Sigma "up to a user-defined
accuracy threshold", keeping its k most significant singular triplets, and
hands the factorisation to a TLR Cholesky whose algorithm it does not print.
The readings taken here (each one a choice, the paper is silent):

* tiles: NT = ceil(n / nb); the last tile holds n - (NT-1) nb points;
* threshold: absolute, spectral norm, per tile: keep singular values
  sigma_t > eps (strictly), so ||A - U V^T||_2 = sigma_{k+1} <= eps; the
  singular values are folded into U (tile = U V^T, U and V have nb x k);
  a tile may get k = 0; k > maxrank raises ``RankError``;
* factorisation: right-looking over k = 0..NT-1:
      L_kk = chol(D_kk)                                  (dense POTRF)
      V_ik <- L_kk^{-1} V_ik            for i > k         (low-rank TRSM)
      D_ii -= U_ik (V_ik^T V_ik) U_ik^T for i > k         (low-rank SYRK)
      for i > j > k:                                      (TLR GEMM)
          X = V_ik^T V_jk
          [U_ij, -U_ik X] = Q1 R1,  [V_ij, U_jk] = Q2 R2  (Householder QR)
          R1 R2^T = W s Z^T, keep s_t > eps               (small SVD)
          U_ij = Q1 W_k diag(s_k),  V_ij = Q2 Z_k
* log|Sigma~| = 2 sum log diag(L_kk); forward solve over the TLR factor
  y_k = L_kk^{-1} (z_k - sum_{j<k} U_kj (V_kj^T y_j)); q = y^T y; l by Eq. (1).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
from scipy.linalg import lapack, solve_triangular

from . import matern as _m
from .dense import NotSPDError


class RankError(ArithmeticError):
    """A tile needed more than ``maxrank`` singular triplets."""

    def __init__(self, i: int, j: int, k: int):
        super().__init__(f"tile ({i},{j}) needs rank {k} > maxrank")
        self.tile = (i, j)
        self.rank = k


def tile_bounds(n: int, nb: int) -> list[tuple[int, int]]:
    nt = (n + nb - 1) // nb
    return [(t * nb, min(n, (t + 1) * nb)) for t in range(nt)]


def compress_svd(A: np.ndarray, eps: float, maxrank: int | None = None,
                 where=(0, 0)) -> tuple[np.ndarray, np.ndarray]:
    """Truncated SVD at absolute eps: A ~ U V^T, U = U_k diag(s_k), V = V_k."""
    W, s, Zt = np.linalg.svd(A, full_matrices=False)
    k = int(np.count_nonzero(s > eps))
    if maxrank is not None and k > maxrank:
        raise RankError(where[0], where[1], k)
    return W[:, :k] * s[:k], np.ascontiguousarray(Zt[:k].T)


@dataclass
class TLRMatrix:
    n: int
    nb: int
    bounds: list
    D: list                       # dense diagonal tiles (lower factor after potrf)
    U: dict = field(default_factory=dict)   # (i, j) i > j -> nb_i x k
    V: dict = field(default_factory=dict)   # (i, j) -> nb_j x k

    @property
    def nt(self) -> int:
        return len(self.bounds)

    def ranks(self) -> np.ndarray:
        R = np.zeros((self.nt, self.nt), dtype=np.int64)
        for (i, j), u in self.U.items():
            R[i, j] = u.shape[1]
        return R


def compress(x, y, theta, nb: int, eps: float, maxrank: int | None = None) -> TLRMatrix:
    """Generate Sigma(theta) tile by tile (Eq. (MaternCov)) and compress the
    strictly-lower tiles by truncated SVD (Section V)."""
    n = len(x)
    bounds = tile_bounds(n, nb)
    D = []
    T = TLRMatrix(n, nb, bounds, D)
    for i, (r0, r1) in enumerate(bounds):
        D.append(_m.covariance(x, y, theta, slice(r0, r1), slice(r0, r1)))
        for j in range(i):
            c0, c1 = bounds[j]
            A = _m.covariance(x, y, theta, slice(r0, r1), slice(c0, c1))
            T.U[(i, j)], T.V[(i, j)] = compress_svd(A, eps, maxrank, (i, j))
    return T


def _recompress(Uh: np.ndarray, Vh: np.ndarray, eps: float):
    Q1, R1 = np.linalg.qr(Uh)
    Q2, R2 = np.linalg.qr(Vh)
    W, s, Zt = np.linalg.svd(R1 @ R2.T)
    k = int(np.count_nonzero(s > eps))
    return Q1 @ (W[:, :k] * s[:k]), Q2 @ Zt[:k].T


def cholesky(T: TLRMatrix, eps: float, maxrank: int | None = None) -> TLRMatrix:
    """Right-looking TLR Cholesky in place (see module docstring)."""
    nt = T.nt
    for k in range(nt):
        c, info = lapack.dpotrf(np.asfortranarray(T.D[k]), lower=1, clean=1)
        if info > 0:
            raise NotSPDError(T.bounds[k][0] + info)
        T.D[k] = c
        for i in range(k + 1, nt):
            T.V[(i, k)] = solve_triangular(c, T.V[(i, k)], lower=True)
        for i in range(k + 1, nt):
            U, V = T.U[(i, k)], T.V[(i, k)]
            T.D[i] = T.D[i] - U @ (V.T @ V) @ U.T
        for i in range(k + 2, nt):
            for j in range(k + 1, i):
                X = T.V[(i, k)].T @ T.V[(j, k)]
                Uh = np.hstack([T.U[(i, j)], -T.U[(i, k)] @ X])
                Vh = np.hstack([T.V[(i, j)], T.U[(j, k)]])
                U, V = _recompress(Uh, Vh, eps)
                if maxrank is not None and U.shape[1] > maxrank:
                    raise RankError(i, j, U.shape[1])
                T.U[(i, j)], T.V[(i, j)] = U, V
    return T


def logdet(T: TLRMatrix) -> float:
    return 2.0 * float(sum(np.sum(np.log(np.diag(d))) for d in T.D))


def forward_solve(T: TLRMatrix, z) -> np.ndarray:
    z = np.asarray(z, dtype=np.float64)
    yv = np.empty_like(z)
    for k, (r0, r1) in enumerate(T.bounds):
        rhs = z[r0:r1].copy()
        for j in range(k):
            c0, c1 = T.bounds[j]
            rhs -= T.U[(k, j)] @ (T.V[(k, j)].T @ yv[c0:c1])
        yv[r0:r1] = solve_triangular(T.D[k], rhs, lower=True)
    return yv


def loglik(x, y, z, theta, nb: int, eps: float, maxrank: int | None = None) -> dict:
    """TLR approximation of Eq. (1): compress, factor, log-det, solve."""
    T = compress(x, y, theta, nb, eps, maxrank)
    ranks0 = T.ranks()
    cholesky(T, eps, maxrank)
    ld = logdet(T)
    w = forward_solve(T, z)
    quad = float(w @ w)
    n = len(z)
    ll = -0.5 * n * math.log(2.0 * math.pi) - 0.5 * ld - 0.5 * quad
    return {"ll": ll, "logdet": ld, "quad": quad, "n": n,
            "ranks_initial": ranks0, "ranks_factor": T.ranks()}
