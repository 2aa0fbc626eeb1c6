"""Pins of the oracle's derivative of the Matérn covariance in the
smoothness nu (oracle/matern.py: dkv_dnu, dmatern_dnu) and of the nu term of
its dense score (oracle/dense.py)."""
import math

import mpmath
import numpy as np
import pytest
from scipy.special import exp1

import synth
from oracle import dense as D
from oracle import matern as M


def test_dkv_dnu_closed_form_at_half():
    # DLMF 10.38.7: dK_nu/dnu at nu = 1/2 equals sqrt(pi / (2x)) E_1(2x) e^x
    x = np.array([1e-3, 0.05, 0.4, 1.0, 2.5, 7.0, 30.0])
    want = np.sqrt(np.pi / (2 * x)) * exp1(2 * x) * np.exp(x)
    np.testing.assert_allclose(M.dkv_dnu(0.5, x), want, rtol=1e-9)


@pytest.mark.parametrize("nu", [0.3, 0.8, 1.0, 1.5, 2.2])
def test_dkv_dnu_against_mpmath(nu):
    mpmath.mp.dps = 40
    for x in (0.01, 0.3, 1.7, 5.0, 20.0):
        want = float(mpmath.diff(lambda v: mpmath.besselk(v, x), nu))
        got = float(M.dkv_dnu(nu, np.array([x]))[0])
        assert abs(got - want) <= 2e-10 * abs(want), (nu, x, got, want)


@pytest.mark.parametrize("nu", [0.5, 1.0, 1.7])
def test_dmatern_dnu_against_mpmath(nu):
    # the whole derivative of C(r; sigma2, beta, nu) in nu, 40-digit mpmath
    mpmath.mp.dps = 40
    s2, beta = 1.3, 0.2
    r = np.array([0.0, 1e-3, 0.05, 0.2, 0.9])

    def c(v, rr):
        u = mpmath.mpf(rr) / beta
        return s2 / (2 ** (v - 1) * mpmath.gamma(v)) * u ** v * mpmath.besselk(v, u)
    got = M.dmatern_dnu(r, s2, beta, nu)
    assert got[0] == 0.0
    for i in range(1, len(r)):
        want = float(mpmath.diff(lambda v: c(v, r[i]), nu))
        # C (log(u/2) - psi) and the K_nu term nearly cancel at small u: the bar
        # is relative to the covariance scale sigma2
        assert abs(got[i] - want) <= 1e-9 * s2, (r[i], got[i], want)


def test_dense_score_nu_central_difference():
    x, y = synth.jittered_subset(250, 3)
    th = (1.1, 0.12, 0.9)
    z = D.sample_z(x, y, th, synth.standard_normal(250, 4))
    g = D.gradient(x, y, z, th)
    h = 1e-5
    lp = D.loglik(x, y, z, (th[0], th[1], th[2] + h))["ll"]
    lm = D.loglik(x, y, z, (th[0], th[1], th[2] - h))["ll"]
    fd = (lp - lm) / (2 * h)
    scale = 0.5 * (abs(g["tr_nu"]) + abs(g["qf_nu"]))
    assert abs(fd - g["dnu"]) <= 1e-6 * scale
    # n = 1: Sigma = sigma^2 for every nu
    g1 = D.gradient(x[:1], y[:1], z[:1], th)
    assert g1["dnu"] == 0.0
