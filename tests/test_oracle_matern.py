"""Pins for oracle.matern: closed forms of Section IV, an independent
quadrature of K_nu, the r -> 0 limit and a finite-difference check of dC/dbeta."""
import math

import numpy as np
import pytest
from scipy import integrate
from scipy.special import k1

from oracle import matern as M

R = np.array([0.0, 1e-9, 1e-4, 0.003, 0.02, 0.1, 0.37, 0.9, 1.41])


@pytest.mark.parametrize("s2,beta", [(1.0, 0.1), (0.7, 0.03), (2.0, 0.3)])
def test_nu_half_is_exponential(s2, beta):
    # Section IV: theta3 = 1/2 gives theta1 exp(-r/theta2).
    np.testing.assert_allclose(M.matern(R, s2, beta, 0.5), s2 * np.exp(-R / beta),
                               rtol=1e-14, atol=0)


@pytest.mark.parametrize("s2,beta", [(1.0, 0.1), (1.3, 0.05)])
def test_nu_three_halves_and_five_halves(s2, beta):
    # Half-integer Matérn closed forms (K_{n+1/2} is elementary).
    u = R / beta
    np.testing.assert_allclose(M.matern(R, s2, beta, 1.5), s2 * (1 + u) * np.exp(-u),
                               rtol=1e-13, atol=0)
    np.testing.assert_allclose(M.matern(R, s2, beta, 2.5),
                               s2 * (1 + u + u * u / 3) * np.exp(-u), rtol=1e-13, atol=0)


def test_nu_one_is_whittle():
    # Section IV: theta3 = 1 gives theta1 (r/theta2) K_1(r/theta2) (k1 is a
    # separate scipy routine from kv).
    s2, beta = 1.2, 0.1
    r = R[R > 0]
    u = r / beta
    np.testing.assert_allclose(M.matern(r, s2, beta, 1.0), s2 * u * k1(u), rtol=1e-13)


@pytest.mark.parametrize("nu", [0.3, 0.75, 1.0, 1.6, 2.2])
def test_general_nu_against_integral_representation(nu):
    # K_nu(x) = int_0^inf exp(-x cosh t) cosh(nu t) dt, evaluated by adaptive
    # quadrature: pins the kv call and the 2^(nu-1) Gamma(nu) normalisation.
    s2, beta = 1.0, 0.2
    for r in [0.01, 0.07, 0.3, 1.1]:
        x = r / beta
        tmax = math.acosh(max(1.0, 800.0 / x)) + 1.0   # integrand < e^-800 beyond
        kint, _ = integrate.quad(lambda t: math.exp(-x * math.cosh(t)) * math.cosh(nu * t),
                                 0, tmax, epsabs=0, epsrel=1e-13, limit=400)
        want = s2 / (2 ** (nu - 1) * math.gamma(nu)) * x ** nu * kint
        assert abs(M.matern(np.array([r]), s2, beta, nu)[0] - want) <= 1e-11 * abs(want)


@pytest.mark.parametrize("nu", [0.5, 1.0, 1.5, 0.8])
def test_zero_distance_limit(nu):
    assert M.matern(np.array([0.0]), 1.7, 0.1, nu)[0] == 1.7
    # continuity: C(r) -> theta1 as r -> 0
    c = M.matern(np.array([1e-10]), 1.7, 0.1, nu)[0]
    assert abs(c - 1.7) < 1e-3


@pytest.mark.parametrize("nu", [0.5, 1.0, 1.5, 0.8])
def test_dbeta_against_central_difference(nu):
    s2, beta = 1.1, 0.12
    r = R[R > 1e-6]
    h = 1e-6 * beta
    fd = (M.matern(r, s2, beta + h, nu) - M.matern(r, s2, beta - h, nu)) / (2 * h)
    an = M.dmatern_dbeta(r, s2, beta, nu)
    np.testing.assert_allclose(an, fd, rtol=2e-7, atol=1e-9)
    assert M.dmatern_dbeta(np.array([0.0]), s2, beta, nu)[0] == 0.0


def test_dbeta_nu_half_closed_form():
    s2, beta = 0.9, 0.07
    np.testing.assert_allclose(M.dmatern_dbeta(R, s2, beta, 0.5),
                               s2 * R / beta ** 2 * np.exp(-R / beta), rtol=1e-13, atol=0)


def test_distances():
    d = M.distances([0, 3], [0, 0], [0], [4])
    np.testing.assert_array_equal(d, [[4.0], [5.0]])
