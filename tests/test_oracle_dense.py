"""Pins for oracle.dense: Eq. (1) closed forms at n = 1, 2, a 50-digit brute
force at n <= 8, invariances, the sigma^2 scaling identity, the chi-square law
of the quadratic form, and the gradient against closed forms and central
differences."""
import math

import mpmath as mp
import numpy as np
import pytest

import synth
from oracle import dense as D
from oracle import matern as M


def _pts(n, seed=3):
    rng = np.random.default_rng(seed)
    return rng.uniform(0, 1, n), rng.uniform(0, 1, n)


def test_n1_closed_form():
    z = np.array([0.83])
    for s2 in (0.5, 1.0, 2.3):
        out = D.loglik([0.2], [0.4], z, (s2, 0.1, 0.5))
        want = -0.5 * math.log(2 * math.pi) - 0.5 * math.log(s2) - z[0] ** 2 / (2 * s2)
        assert abs(out["ll"] - want) < 1e-15 * abs(want) + 1e-15


def test_n2_closed_form():
    x, y = [0.1, 0.13], [0.2, 0.16]
    z = np.array([0.7, -1.1])
    s2, beta = 1.4, 0.1
    r = math.hypot(x[1] - x[0], y[1] - y[0])
    rho = math.exp(-r / beta)
    det = s2 * s2 * (1 - rho * rho)
    q = (z[0] ** 2 - 2 * rho * z[0] * z[1] + z[1] ** 2) / (s2 * (1 - rho * rho))
    want = -math.log(2 * math.pi) - 0.5 * math.log(det) - 0.5 * q
    out = D.loglik(x, y, z, (s2, beta, 0.5))
    assert abs(out["ll"] - want) < 1e-13 * abs(want)
    assert abs(out["quad"] - q) < 1e-13 * q


@pytest.mark.parametrize("n,nu", [(5, 0.5), (8, 1.0), (7, 1.5)])
def test_bruteforce_mpmath(n, nu):
    # 50-digit determinant and inverse with mpmath's own Bessel K.
    mp.mp.dps = 50
    x, y = _pts(n, seed=n)
    z = np.random.default_rng(n).standard_normal(n)
    s2, beta = 1.3, 0.15
    S = mp.matrix(n, n)
    for a in range(n):
        for b in range(n):
            r = mp.sqrt((mp.mpf(x[a]) - x[b]) ** 2 + (mp.mpf(y[a]) - y[b]) ** 2)
            if r == 0:
                S[a, b] = mp.mpf(s2)
            else:
                u = r / beta
                S[a, b] = s2 / (2 ** (mp.mpf(nu) - 1) * mp.gamma(nu)) * u ** nu * mp.besselk(nu, u)
    det = mp.det(S)
    zz = mp.matrix([mp.mpf(v) for v in z])
    q = (zz.T * mp.lu_solve(S, zz))[0]
    want = -n / mp.mpf(2) * mp.log(2 * mp.pi) - mp.log(det) / 2 - q / 2
    out = D.loglik(x, y, z, (s2, beta, nu))
    assert abs(out["ll"] - float(want)) < 1e-10 * abs(float(want))
    assert abs(out["logdet"] - float(mp.log(det))) < 1e-10 * max(1.0, abs(float(mp.log(det))))


def test_permutation_invariance():
    x, y = _pts(300)
    z = np.random.default_rng(0).standard_normal(300)
    th = (1.0, 0.1, 0.5)
    a = D.loglik(x, y, z, th)["ll"]
    p = np.random.default_rng(9).permutation(300)
    b = D.loglik(x[p], y[p], z[p], th)["ll"]
    assert abs(a - b) < 1e-10 * abs(a)


def test_sigma2_scaling_identity():
    # Sigma(c s2) = c Sigma(s2): l(c s2) = l(s2) - n/2 log c - q/2 (1/c - 1)
    x, y = _pts(250)
    z = np.random.default_rng(2).standard_normal(250)
    base = D.loglik(x, y, z, (1.0, 0.08, 1.0))
    for c in (0.3, 2.5):
        got = D.loglik(x, y, z, (c, 0.08, 1.0))["ll"]
        want = base["ll"] - 250 / 2 * math.log(c) - 0.5 * base["quad"] * (1 / c - 1)
        assert abs(got - want) < 1e-10 * abs(want)


def test_quadratic_form_chi_square():
    # z = L eps  =>  q = eps^T eps ~ chi^2_n
    n = 900
    x, y = synth.jittered_grid(30, seed=0)
    eps = synth.standard_normal(n, seed=1)
    th = (1.0, 0.1, 0.5)
    z = D.sample_z(x, y, th, eps)
    q = D.loglik(x, y, z, th)["quad"]
    assert abs(q - float(eps @ eps)) < 1e-8 * q
    assert abs(q - n) < 6 * math.sqrt(2 * n)


def test_not_spd_reports_pivot():
    with pytest.raises(D.NotSPDError) as e:
        D.loglik([0.1, 0.5], [0.1, 0.5], np.ones(2), (-1.0, 0.1, 0.5))
    assert e.value.info == 1


def test_gradient_sigma2_closed_form():
    x, y = _pts(200)
    z = np.random.default_rng(4).standard_normal(200)
    for th in [(1.0, 0.1, 0.5), (0.6, 0.05, 1.0)]:
        g = D.gradient(x, y, z, th)
        want = (g["quad"] - 200) / (2 * th[0])
        assert abs(g["dsigma2"] - want) < 1e-9 * max(1.0, abs(want))


@pytest.mark.parametrize("th", [(1.0, 0.1, 0.5), (0.7, 0.05, 1.0), (1.2, 0.2, 1.5)])
def test_gradient_beta_central_difference(th):
    x, y = synth.jittered_grid(17, seed=0)
    z = D.sample_z(x, y, th, np.random.default_rng(5).standard_normal(289))
    g = D.gradient(x, y, z, th)
    h = 1e-5 * th[1]
    lp = D.loglik(x, y, z, (th[0], th[1] + h, th[2]))["ll"]
    lm = D.loglik(x, y, z, (th[0], th[1] - h, th[2]))["ll"]
    fd = (lp - lm) / (2 * h)
    assert abs(g["dbeta"] - fd) < 1e-6 * max(1.0, abs(fd))


def test_gradient_n1_and_n2():
    # n = 1: Sigma = sigma2 does not depend on beta.
    g1 = D.gradient([0.3], [0.3], np.array([0.4]), (1.0, 0.1, 0.5))
    assert g1["dbeta"] == 0.0
    # n = 2, nu = 1/2: rho = exp(-r/beta), drho/dbeta = r/beta^2 rho.
    x, y = [0.1, 0.16], [0.2, 0.23]
    z = np.array([0.9, 0.4])
    s2, beta = 1.0, 0.1
    r = math.hypot(0.06, 0.03)
    rho = math.exp(-r / beta)
    Qz = z[0] ** 2 - 2 * rho * z[0] * z[1] + z[1] ** 2
    dl_drho = rho / (1 - rho ** 2) - 0.5 / s2 * (-2 * z[0] * z[1] * (1 - rho ** 2) + 2 * rho * Qz) / (1 - rho ** 2) ** 2
    want = dl_drho * r / beta ** 2 * rho
    g2 = D.gradient(x, y, z, (s2, beta, 0.5))
    assert abs(g2["dbeta"] - want) < 1e-10 * abs(want)


def test_covariance_symmetric_positive():
    x, y = synth.jittered_grid(12, seed=0)
    S = M.covariance(x, y, (1.0, 0.1, 1.0))
    assert np.array_equal(S, S.T)
    assert np.all(np.diag(S) == 1.0)
    assert np.linalg.eigvalsh(S).min() > 0
