"""Pins of the tiled dense oracle (oracle/tiled.py), which produces the stored
expected values at n = 40,000 and 102,400.  It must equal the plain dense
oracle (itself pinned by closed forms and brute force) wherever both fit,
for any tile size including ragged ones, and meet the closed forms on its own.
"""
import math

import numpy as np
import pytest

import synth
from oracle import dense as D
from oracle import matern as M
from oracle import ordering as O
from oracle import tiled as T
from oracle import tlr as OT


def _field(n, seed, th):
    x, y = synth.jittered_subset(n, seed)
    p = O.morton_order(x, y)
    x, y = x[p].copy(), y[p].copy()
    z = D.sample_z(x, y, th, synth.standard_normal(n, seed + 1))
    return x, y, z


@pytest.mark.parametrize("nb", [700, 97, 256, 1])
def test_tiled_loglik_equals_dense(nb):
    th = (1.0, 0.1, 1.0)
    x, y, z = _field(700 if nb > 1 else 60, 4, th)
    r = D.loglik(x, y, z, th)
    t = T.loglik(x, y, z, th, nb=nb)
    for k in ("ll", "logdet", "quad"):
        assert abs(t[k] - r[k]) <= 1e-12 * abs(r[k]), k


def test_tiled_gradient_equals_dense():
    th = (1.2, 0.07, 1.5)
    x, y, z = _field(500, 5, th)
    r = D.gradient(x, y, z, th)
    t = T.gradient(x, y, z, th, nb=128)
    for k in ("ll", "logdet", "quad", "tr_beta", "qf_beta"):
        assert abs(t[k] - r[k]) <= 1e-11 * abs(r[k]), k
    for k in ("dsigma2", "dbeta"):
        scale = 0.5 * (abs(r["tr_beta"]) + abs(r["qf_beta"]))
        assert abs(t[k] - r[k]) <= 1e-11 * scale, k


def test_tiled_closed_forms_n1_n2():
    s2, beta, nu = 1.4, 0.2, 0.5
    x, y, z = np.array([0.3]), np.array([0.6]), np.array([0.9])
    t = T.gradient(x, y, z, (s2, beta, nu), nb=1)
    assert abs(t["ll"] - (-0.5 * math.log(2 * math.pi) - 0.5 * math.log(s2) - z[0] ** 2 / (2 * s2))) <= 1e-15
    assert abs(t["dsigma2"] - (z[0] ** 2 / s2 - 1) / (2 * s2)) <= 1e-15
    assert t["dbeta"] == 0.0
    x, y, z = np.array([0.1, 0.25]), np.array([0.3, 0.2]), np.array([0.5, -1.2])
    r = math.hypot(x[0] - x[1], y[0] - y[1])
    rho = math.exp(-r / beta)   # nu = 1/2: exponential
    det = s2 * s2 * (1 - rho * rho)
    q = (z[0] ** 2 - 2 * rho * z[0] * z[1] + z[1] ** 2) / (s2 * (1 - rho * rho))
    for nb in (1, 2):
        t = T.loglik(x, y, z, (s2, beta, nu), nb=nb)
        assert abs(t["logdet"] - math.log(det)) <= 1e-14
        assert abs(t["quad"] - q) <= 1e-14 * q
        assert abs(t["ll"] - (-math.log(2 * math.pi) - 0.5 * math.log(det) - 0.5 * q)) <= 1e-14


def test_tiled_inverse_against_brute_force():
    th = (1.0, 0.1, 0.5)
    x, y, _ = _field(300, 6, th)
    L = T.cholesky_tiles(T.covariance_tiles(x, y, th, 70))
    S = T.inverse_tiles(L).to_dense()
    A = M.covariance(x, y, th)
    np.testing.assert_allclose(S @ A, np.eye(300), atol=1e-9)
    np.testing.assert_allclose(S, np.linalg.inv(A), rtol=0, atol=1e-9 * np.abs(S).max())


def test_tiled_factor_matches_lapack_and_sample():
    th = (1.0, 0.1, 1.0)
    x, y, _ = _field(400, 7, th)
    L = T.cholesky_tiles(T.covariance_tiles(x, y, th, 96)).to_dense()
    Lr = D.cholesky_lower(M.covariance(x, y, th))
    np.testing.assert_allclose(np.tril(L), Lr, rtol=0, atol=1e-13)
    e = synth.standard_normal(400, 8)
    np.testing.assert_allclose(T.sample_z(x, y, th, e, nb=96), D.sample_z(x, y, th, e), rtol=0, atol=1e-13)


def test_tiled_equals_tlr_at_eps_zero():
    # the TLR oracle with nothing truncated is the dense factor (Section V)
    th = (1.0, 0.1, 0.5)
    x, y, z = _field(600, 9, th)
    a = T.loglik(x, y, z, th, nb=150)
    b = OT.loglik(x, y, z, th, nb=150, eps=0.0, maxrank=150)
    assert abs(a["ll"] - b["ll"]) <= 1e-11 * abs(a["ll"])


def test_tiled_not_spd_global_row():
    x, y = synth.jittered_subset(50, 0)
    with pytest.raises(D.NotSPDError) as e:
        T.loglik(x, y, np.ones(50), (-1.0, 0.1, 0.5), nb=16)
    assert e.value.info == 1
    # a diagonal matrix with one negative entry, global row 38 (tile 2 of 16)
    A = np.eye(50)
    A[37, 37] = -1.0
    Lt = T.LowerTiles(50, 16)
    for i in range(Lt.nt):
        for j in range(i + 1):
            Lt.t[i][j] = np.asfortranarray(A[Lt.sl(i), Lt.sl(j)])
    with pytest.raises(D.NotSPDError) as e:
        T.cholesky_tiles(Lt)
    assert e.value.info == 38
