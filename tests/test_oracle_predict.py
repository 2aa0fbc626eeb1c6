"""Pins of the oracle's kriging prediction (oracle/predict.py, Section III
Eqs. (pred2)-(pred3)) and of its great-circle distance (Section IV,
Eq. (gcd)), against facts that do not depend on their code."""
import math

import numpy as np

import synth
from oracle import dense as D
from oracle import matern as M
from oracle import predict as PR


def _field(n, seed, th):
    x, y = synth.jittered_subset(n, seed)
    z = D.sample_z(x, y, th, synth.standard_normal(n, seed + 1))
    return x, y, z


def test_prediction_equals_gaussian_conditioning_via_precision():
    # the conditional mean of a zero-mean Gaussian is -P11^{-1} P12 z2 with P
    # the inverse of the joint covariance (block inverse identity)
    th = (1.3, 0.15, 1.0)
    x, y, z = _field(300, 3, th)
    xn, yn = np.array([0.11, 0.52, 0.93, 0.5]), np.array([0.07, 0.48, 0.61, 0.5001])
    pred, var = PR.predict(x, y, z, xn, yn, th, variance=True)
    X, Y = np.concatenate([xn, x]), np.concatenate([yn, y])
    Pm = np.linalg.inv(M.covariance(X, Y, th))
    m = len(xn)
    P11, P12 = Pm[:m, :m], Pm[:m, m:]
    np.testing.assert_allclose(pred, -np.linalg.solve(P11, P12 @ z), rtol=1e-9, atol=1e-10)
    np.testing.assert_allclose(var, np.diag(np.linalg.inv(P11)), rtol=1e-8, atol=1e-12)


def test_prediction_interpolates_observations():
    # no nugget: at an observed location the predictor returns the
    # observation and the conditional variance vanishes
    th = (1.0, 0.1, 0.5)
    x, y, z = _field(200, 4, th)
    idx = np.array([0, 17, 199])
    pred, var = PR.predict(x, y, z, x[idx], y[idx], th, variance=True)
    np.testing.assert_allclose(pred, z[idx], rtol=1e-9, atol=1e-9)
    assert np.all(np.abs(var) <= 1e-9)


def test_prediction_one_observation_closed_form():
    s2, beta, nu = 2.0, 0.2, 0.5
    x, y, z = np.array([0.3]), np.array([0.4]), np.array([1.7])
    xn, yn = np.array([0.5, 5.0]), np.array([0.4, 5.0])
    rho = np.exp(-np.hypot(xn - x[0], yn - y[0]) / beta)
    pred, var = PR.predict(x, y, z, xn, yn, (s2, beta, nu), variance=True)
    np.testing.assert_allclose(pred, rho * z[0], rtol=1e-14)
    np.testing.assert_allclose(var, s2 * (1 - rho ** 2), rtol=1e-14)


def test_mse():
    assert PR.mse([1.0, 2.0, 4.0], [1.0, 3.0, 2.0]) == (0 + 1 + 4) / 3


def test_great_circle_against_vincenty_and_known_values():
    r = M.EARTH_RADIUS_KM
    rng = np.random.default_rng(5)
    lon = rng.uniform(-180, 180, 40)
    lat = rng.uniform(-89, 89, 40)
    # nearby points too
    lon = np.concatenate([lon, lon[:10] + 1e-4])
    lat = np.concatenate([lat, lat[:10] - 2e-4])
    d = M.distances(lon, lat, lon, lat, "great_circle")
    p1, p2 = np.radians(lat)[:, None], np.radians(lat)[None, :]
    dl = np.radians(lon)[None, :] - np.radians(lon)[:, None]
    num = np.hypot(np.cos(p2) * np.sin(dl), np.cos(p1) * np.sin(p2) - np.sin(p1) * np.cos(p2) * np.cos(dl))
    den = np.sin(p1) * np.sin(p2) + np.cos(p1) * np.cos(p2) * np.cos(dl)
    vin = r * np.arctan2(num, den)
    np.testing.assert_allclose(d, vin, rtol=1e-11, atol=1e-9)
    assert np.all(np.diag(d) == 0.0)
    np.testing.assert_allclose(d, d.T, rtol=1e-14, atol=0)
    # a quarter meridian and a quarter of the equator: pi r / 2
    q = M.distances([0.0, 0.0], [0.0, 0.0], [0.0, 90.0], [90.0, 0.0], "great_circle")
    np.testing.assert_allclose([q[0, 0], q[1, 1]], [math.pi * r / 2] * 2, rtol=1e-15)
    # antipodes: pi r
    a = M.distances([10.0], [20.0], [-170.0], [-20.0], "great_circle")
    np.testing.assert_allclose(a[0, 0], math.pi * r, rtol=1e-12)
