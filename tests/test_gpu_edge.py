"""Degenerate sizes and the split-K GEMM path, through the C-ABI.

* n = 1 and n = 2 against their closed forms (Eq. (1) with a 1 x 1 and a
  2 x 2 Sigma): l, and the score (dl/dbeta = 0 at n = 1);
* the split-K path of the MFMA GEMM (long inner dimension, few output tiles)
  is reached by a dense factorisation whose last tile columns have K >= 2048
  and a small output grid; the library counts such launches, and the result
  matches the oracle.
"""
import math

import numpy as np
import pytest

from oracle import dense as D

from gpu_util import field, log, to_dev

pytestmark = pytest.mark.gpu


def _closed_forms(x, y, z, th):
    s2, beta, nu = th
    n = len(z)
    if n == 1:
        ll = -0.5 * math.log(2 * math.pi) - 0.5 * math.log(s2) - z[0] ** 2 / (2 * s2)
        return ll, ((z[0] ** 2 / s2 - 1.0) / (2 * s2), 0.0)
    assert nu == 1.5
    r = math.hypot(x[0] - x[1], y[0] - y[1])
    u = r / beta
    rho = (1.0 + u) * math.exp(-u)          # Matérn correlation at nu = 3/2
    drho = u * u * math.exp(-u) / beta      # its derivative in beta
    det = s2 * s2 * (1 - rho * rho)
    q = (z[0] ** 2 - 2 * rho * z[0] * z[1] + z[1] ** 2) / (s2 * (1 - rho * rho))
    ll = -math.log(2 * math.pi) - 0.5 * math.log(det) - 0.5 * q
    # dl/drho of the bivariate normal, times drho/dbeta
    a = z[0] * z[0] + z[1] * z[1]
    b = z[0] * z[1]
    dq = (-2 * b * (1 - rho * rho) + 2 * rho * (a - 2 * rho * b)) / (s2 * (1 - rho * rho) ** 2)
    dll_drho = rho / (1 - rho * rho) - 0.5 * dq
    return ll, ((q - 2.0) / (2 * s2), dll_drho * drho)


@pytest.mark.parametrize("mode", ["dense", "tlr"])
@pytest.mark.parametrize("n", [1, 2])
def test_tiny_n_closed_forms(n, mode):
    import paper_1804_09137_amd as P
    th = (1.3, 0.2, 0.5) if n == 1 else (0.8, 0.3, 1.5)
    x = np.array([0.21, 0.37])[:n]
    y = np.array([0.44, 0.29])[:n]
    z = np.array([0.7, -1.1])[:n]
    ll_c, g_c = _closed_forms(x, y, z, th)
    xd, yd, zd = to_dev(x, y, z)
    h = P.Handle(n, 32, mode=mode, tol=1e-9, want_grad=True)
    ll, g = h.loglik_grad(xd, yd, zd, th)
    h2 = P.Handle(n, 32, mode=mode, tol=1e-9)
    h2.generate(xd, yd, th)
    h2.potrf()
    ll2, _, _ = h2.loglik(zd)
    log(f"n={n} {mode}: ll {ll!r} {ll2!r} closed {ll_c!r}; grad {g} closed {g_c}")
    for v in (ll, ll2):
        assert abs(v - ll_c) <= 1e-14 * max(1.0, abs(ll_c))
    assert abs(g[0] - g_c[0]) <= 1e-14 * max(1.0, abs(g_c[0]))
    assert abs(g[1] - g_c[1]) <= 1e-13 * max(1.0, abs(g_c[1]))
    if n == 1:
        assert g[1] == 0.0


def test_split_k_gemm_path():
    import paper_1804_09137_amd as P
    n, nb = 4096, 512
    th = (1.0, 0.1, 0.5)
    x, y, z = field(n, 21, th)
    ref = D.gradient(x, y, z, th)
    xd, yd, zd = to_dev(x, y, z)
    h = P.Handle(n, nb, mode="dense", want_grad=True)
    ll, g = h.loglik_grad(xd, yd, zd, th)
    i = h.info()
    log(f"split-K launches {i.splitk_launches}; ll {ll} vs {ref['ll']}; dbeta {g[1]} vs {ref['dbeta']}")
    assert i.splitk_launches > 0
    assert abs(ll - ref["ll"]) <= 1e-9 * abs(ref["ll"])
    scale = 0.5 * (abs(ref["tr_beta"]) + abs(ref["qf_beta"]))
    assert abs(g[1] - ref["dbeta"]) <= 1e-8 * scale
