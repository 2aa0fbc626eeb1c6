"""Kriging prediction (Section III, Eqs. (pred2)-(pred3)) and the
great-circle distance (Section IV, Eq. (gcd)) through the C-ABI, against the
CPU oracle (oracle/predict.py, oracle/matern.py).

Tolerances: dense FP64 prediction within 1e-9 of the oracle relative to
max|z|; TLR within 100 eps of it (the factor's error reaches the prediction
through Sigma_22^{-1}); conditional variances likewise relative to sigma^2.
"""
import numpy as np
import pytest

import synth
from oracle import dense as D
from oracle import matern as M
from oracle import predict as PR
from oracle import ordering as O

from gpu_util import log, to_dev

pytestmark = pytest.mark.gpu


def _train_test(n, m, seed, th, metric="euclid", box=None):
    """n + m jittered points (Morton order over all of them), z of the whole
    set from the oracle's dense factor; m random points held out."""
    x, y = synth.jittered_subset(n + m, seed)
    if box is not None:
        x = box[0] + (box[1] - box[0]) * x
        y = box[2] + (box[3] - box[2]) * y
    p = O.morton_order(x, y)
    x, y = x[p].copy(), y[p].copy()
    L = D.cholesky_lower(M.covariance(x, y, th, metric=metric))
    z = L @ synth.standard_normal(n + m, seed + 1)
    test = np.sort(np.random.default_rng(seed + 2).choice(n + m, m, replace=False))
    train = np.setdiff1d(np.arange(n + m), test)
    return x[train], y[train], z[train], x[test], y[test], z[test]


@pytest.mark.parametrize("mode,eps", [("dense", 0.0), ("tlr", 1e-9), ("tlr", 1e-7)])
def test_predict_matches_oracle(mode, eps):
    import paper_1804_09137_amd as P
    n, m, nb = 3000, 100, 256
    th = (1.0, 0.1, 0.5)
    x, y, z, xn, yn, zt = _train_test(n, m, 31, th)
    ref, rvar = PR.predict(x, y, z, xn, yn, th, variance=True)
    h = P.Handle(n, nb, mode=mode, tol=max(eps, 1e-9), maxrank=128)
    xd, yd, zd, xnd, ynd = to_dev(x, y, z, xn, yn)
    h.generate(xd, yd, th)
    h.potrf()
    pred, var = h.predict(zd, xnd, ynd, variance=True)
    pred, var = pred.cpu().numpy(), var.cpu().numpy()
    zs = np.abs(z).max()
    tol = 1e-9 if mode == "dense" else 100 * eps
    e_p = np.abs(pred - ref).max() / zs
    e_v = np.abs(var - rvar).max() / th[0]
    log(f"{mode} eps={eps}: pred err {e_p:.2e}, var err {e_v:.2e}; MSE {PR.mse(pred, zt):.4f} "
        f"(oracle {PR.mse(ref, zt):.4f})")
    assert e_p <= tol
    assert e_v <= tol
    # prediction-only call gives the same values
    pred2 = h.predict(zd, xnd, ynd).cpu().numpy()
    assert np.array_equal(pred2, pred)


def test_predict_interpolates_and_edge_sizes():
    import paper_1804_09137_amd as P
    n, nb = 1500, 160
    th = (1.3, 0.1, 1.5)
    x, y, z, _, _, _ = _train_test(n, 1, 41, th)
    h = P.Handle(n, nb, tol=1e-10, maxrank=80)
    xd, yd, zd = to_dev(x, y, z)
    h.generate(xd, yd, th)
    h.potrf()
    idx = np.array([0, 700, n - 1])
    xnd, ynd = to_dev(x[idx], y[idx])
    pred, var = h.predict(zd, xnd, ynd, variance=True)
    np.testing.assert_allclose(pred.cpu().numpy(), z[idx], rtol=0, atol=1e-6 * np.abs(z).max())
    assert np.all(np.abs(var.cpu().numpy()) <= 1e-6 * th[0])
    # m = 0 is a no-op; before potrf the call is an error
    import torch
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    assert h.predict(zd, e, e).numel() == 0
    h2 = P.Handle(n, nb, tol=1e-10)
    h2.generate(xd, yd, th)
    with pytest.raises(P.TLRError):
        h2.predict(zd, xnd, ynd)


def test_prediction_mse_by_range():
    # held-out prediction error for weak / medium / strong correlation
    # (Section VIII-D uses beta = 0.03, 0.1, 0.3 and 100 missing values);
    # GPU TLR and oracle MSE agree, and the error falls as the range grows
    import paper_1804_09137_amd as P
    n, m, nb, eps = 4000, 100, 320, 1e-9
    out = []
    for beta in (0.03, 0.1, 0.3):
        th = (1.0, beta, 0.5)
        x, y, z, xn, yn, zt = _train_test(n, m, 51, th)
        ref = PR.predict(x, y, z, xn, yn, th)
        h = P.Handle(n, nb, tol=eps, maxrank=160)
        xd, yd, zd, xnd, ynd = to_dev(x, y, z, xn, yn)
        h.generate(xd, yd, th)
        h.potrf()
        pred = h.predict(zd, xnd, ynd).cpu().numpy()
        a, b = PR.mse(pred, zt), PR.mse(ref, zt)
        log(f"beta={beta}: MSE GPU TLR {a:.5f}, oracle {b:.5f}")
        assert abs(a - b) <= 1e-6 * b
        out.append(a)
        h.close()
    assert out[0] > out[1] > out[2]


BOX = (30.0, 60.0, 10.0, 40.0)   # longitude and latitude ranges, degrees


def test_great_circle_covariance_block():
    import paper_1804_09137_amd as P
    n = 600
    th = (1.0, 300.0, 1.0)   # range in km
    x, y = synth.jittered_subset(n, 61)
    x = BOX[0] + (BOX[1] - BOX[0]) * x
    y = BOX[2] + (BOX[3] - BOX[2]) * y
    h = P.Handle(n, 128, tol=1e-9, metric="great_circle")
    xd, yd = to_dev(x, y)
    h.generate(xd, yd, th)
    C = h.covariance_block(0, n, 0, n).cpu().numpy()
    want = M.covariance(x, y, th, metric="great_circle")
    np.testing.assert_allclose(C, want, rtol=2e-13, atol=1e-300)
    dC = h.covariance_block(10, 200, 30, 300, deriv=True).cpu().numpy()
    dwant = M.covariance_dbeta(x, y, th, slice(10, 210), slice(30, 330), metric="great_circle")
    np.testing.assert_allclose(dC, dwant, rtol=5e-13, atol=1e-300)


@pytest.mark.parametrize("mode,eps", [("dense", 0.0), ("tlr", 1e-8)])
def test_great_circle_loglik_and_score(mode, eps):
    import paper_1804_09137_amd as P
    n, nb = 2500, 256
    th = (1.0, 250.0, 0.5)
    x, y, z, _, _, _ = _train_test(n, 1, 71, th, metric="great_circle", box=BOX)
    # the oracle's dense score, with the great-circle covariance
    S = M.covariance(x, y, th, metric="great_circle")
    L = D.cholesky_lower(S)
    w = np.linalg.solve(L, z)
    ld = 2 * np.sum(np.log(np.diag(L)))
    ll_ref = -0.5 * n * np.log(2 * np.pi) - 0.5 * ld - 0.5 * w @ w
    Si = np.linalg.inv(S)
    a = Si @ z
    dB = M.covariance_dbeta(x, y, th, metric="great_circle")
    db_ref = -0.5 * np.sum(Si * dB) + 0.5 * a @ dB @ a
    h = P.Handle(n, nb, mode=mode, tol=max(eps, 1e-9), want_grad=True, metric="great_circle")
    xd, yd, zd = to_dev(x, y, z)
    ll, g = h.loglik_grad(xd, yd, zd, th)
    scale = 0.5 * (abs(np.sum(Si * dB)) + abs(a @ dB @ a))
    log(f"great circle {mode}: ll {ll:.10g} vs {ll_ref:.10g}; dbeta {g[1]:.8g} vs {db_ref:.8g}")
    if mode == "dense":
        assert abs(ll - ll_ref) <= 1e-9 * abs(ll_ref)
        assert abs(g[1] - db_ref) <= 1e-8 * scale
    else:
        assert abs(ll - ll_ref) <= 10 * eps * abs(ll_ref)
        assert abs(g[1] - db_ref) <= 100 * eps * scale
