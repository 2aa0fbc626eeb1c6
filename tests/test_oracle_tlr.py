"""Pins for oracle.tlr: the SVD truncation theorem on exact low-rank tiles,
reduction to the dense result when nothing is truncated, error shrinking with
the threshold, and the factor's residual against Sigma."""
import numpy as np
import pytest

import synth
from oracle import dense as D
from oracle import matern as M
from oracle import ordering as O
from oracle import tlr as T


def _field(m, seed=0, th=(1.0, 0.1, 0.5)):
    x, y = synth.jittered_grid(m, seed)
    p = O.morton_order(x, y)
    x, y = x[p], y[p]
    z = D.sample_z(x, y, th, synth.standard_normal(m * m, seed + 1))
    return x, y, z


def test_compress_exact_rank_tile():
    rng = np.random.default_rng(0)
    A = rng.standard_normal((120, 5)) @ rng.standard_normal((5, 90))
    U, V = T.compress_svd(A, 1e-9)
    assert U.shape == (120, 5) and V.shape == (90, 5)
    assert np.linalg.norm(A - U @ V.T, 2) < 1e-12 * np.linalg.norm(A, 2)


def test_compress_error_bound_and_monotone_rank():
    x, y = synth.jittered_grid(20, seed=0)
    A = M.covariance(x, y, (1.0, 0.1, 0.5), slice(0, 200), slice(200, 400))
    s = np.linalg.svd(A, compute_uv=False)
    last = None
    for eps in (1e-3, 1e-5, 1e-7, 1e-9):
        U, V = T.compress_svd(A, eps)
        k = U.shape[1]
        assert np.linalg.norm(A - U @ V.T, 2) <= eps * (1 + 1e-6) + 1e-13
        assert k == int(np.sum(s > eps))
        if last is not None:
            assert k >= last
        last = k


def test_rank_overflow_raises():
    x, y = synth.jittered_grid(20, seed=0)
    with pytest.raises(T.RankError):
        T.compress(x, y, (1.0, 0.1, 0.5), nb=100, eps=1e-12, maxrank=2)


def test_no_truncation_equals_dense():
    x, y, z = _field(24)          # n = 576, 4 tiles of 150 (+ragged 126)
    th = (1.0, 0.1, 0.5)
    dense = D.loglik(x, y, z, th)
    tl = T.loglik(x, y, z, th, nb=150, eps=0.0)
    assert abs(tl["ll"] - dense["ll"]) < 1e-10 * abs(dense["ll"])
    assert abs(tl["logdet"] - dense["logdet"]) < 1e-10 * abs(dense["logdet"])


def test_error_shrinks_with_threshold():
    x, y, z = _field(30)          # n = 900, nb = 200 -> 5 tiles, ragged 100
    th = (1.0, 0.1, 0.5)
    ref = D.loglik(x, y, z, th)["ll"]
    errs = [abs(T.loglik(x, y, z, th, nb=200, eps=e)["ll"] - ref) for e in (1e-3, 1e-6, 1e-9)]
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-8 * abs(ref)


def test_factor_residual_is_order_eps():
    x, y, _ = _field(20)
    th = (1.0, 0.1, 1.0)
    eps = 1e-8
    F = T.cholesky(T.compress(x, y, th, 100, eps), eps)
    n = len(x)
    L = np.zeros((n, n))
    for i, (r0, r1) in enumerate(F.bounds):
        L[r0:r1, r0:r1] = F.D[i]
        for j in range(i):
            c0, c1 = F.bounds[j]
            L[r0:r1, c0:c1] = F.U[(i, j)] @ F.V[(i, j)].T
    S = M.covariance(x, y, th)
    assert np.max(np.abs(L @ L.T - S)) < 50 * eps


def test_config0_accuracy():
    # n = 1600 (40 x 40), nb = 320, eps = 1e-9, maxrank 160
    x, y, z = _field(40)
    th = (1.0, 0.1, 0.5)
    ref = D.loglik(x, y, z, th)["ll"]
    tl = T.loglik(x, y, z, th, nb=320, eps=1e-9, maxrank=160)
    assert abs(tl["ll"] - ref) <= 10 * 1e-9 * abs(ref)
    assert tl["ranks_initial"].max() <= 160
