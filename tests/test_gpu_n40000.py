"""GPU parity at the n = 40,000 workloads (200 x 200 jittered grid, Morton
order, tile 560 = 71 full tiles and a ragged one of 240; Section VIII-D runs
its Monte Carlo study at this size).

Expected values come from ``tests/golden/n40000.json``, written by
``tests/golden/make_golden.py`` with the CPU oracle's tiled dense
log-likelihood and score (``oracle/tiled.py``); the measurement vector z is
``tests/golden/n40000_z.npy`` from the same script (z = L eps of the field
at theta_true = (1, 0.1, 0.5)).

Tolerances: dense FP64 within 1e-9 |l|; TLR within 10 eps |l|, or, where the
oracle's own exact-SVD TLR at the same eps (``tests/golden/n40000_tlr_EPS.json``,
same script) is itself further than that from the dense value (smooth,
strongly correlated fields), within twice the oracle TLR's error -- the rule
the smaller ill-conditioned parity case uses.  The metric's gate
|dl| <= 1e-6 |l| is reported per (theta, eps).
"""
from __future__ import annotations

import functools
import hashlib
import json
import os

import numpy as np
import pytest

import synth
from oracle import ordering as O

from gpu_util import log, to_dev

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = os.path.join(HERE, "golden", "n40000.json")
NB = 560


@functools.lru_cache(maxsize=1)
def _case():
    import paper_1804_09137_amd as P
    with open(GOLD) as f:
        g = json.load(f)
    x, y = synth.jittered_grid(g["grid"], g["loc_seed"])
    p = P.morton_order(x, y)
    assert np.array_equal(p, O.morton_order(x, y))
    x, y = x[p].copy(), y[p].copy()
    z = np.load(os.path.join(HERE, "golden", "n40000_z.npy"))
    assert hashlib.sha256(z.tobytes()).hexdigest() == g["z_sha256"]
    return g, x, y, z


def _dev():
    g, x, y, z = _case()
    return to_dev(x, y, z)


def _records():
    with open(GOLD) as f:
        return json.load(f)["loglik"]


@pytest.fixture(scope="module")
def dense_handle():
    import paper_1804_09137_amd as P
    h = P.Handle(40000, NB, mode="dense")
    yield h
    h.close()


@pytest.mark.parametrize("rec", _records(), ids=lambda r: f"b{r['theta'][1]}-nu{r['theta'][2]}")
def test_dense_loglik_n40000(rec, dense_handle):
    th = tuple(rec["theta"])
    log(f"dense n=40000 theta={th}")
    xd, yd, zd = _dev()
    dense_handle.generate(xd, yd, th)
    dense_handle.potrf()
    ll, ld, q = dense_handle.loglik(zd)
    log(f"  ll={ll:.15g} oracle={rec['ll']:.15g} rel={abs(ll - rec['ll']) / abs(rec['ll']):.2e}")
    assert abs(ll - rec["ll"]) <= 1e-9 * abs(rec["ll"])
    assert abs(ld - rec["logdet"]) <= 1e-9 * abs(rec["logdet"])
    assert abs(q - rec["quad"]) <= 1e-9 * abs(rec["quad"])


@pytest.mark.parametrize("eps", [1e-5, 1e-7, 1e-9])
@pytest.mark.parametrize("rec", _records(), ids=lambda r: f"b{r['theta'][1]}-nu{r['theta'][2]}")
def test_tlr_loglik_n40000(rec, eps):
    import paper_1804_09137_amd as P
    th = tuple(rec["theta"])
    xd, yd, zd = _dev()
    log(f"tlr n=40000 theta={th} eps={eps}")
    h = P.Handle(40000, NB, tol=eps)
    h.generate(xd, yd, th)
    h.potrf()
    ll, _, _ = h.loglik(zd)
    i = h.info()
    rel = abs(ll - rec["ll"]) / abs(rec["ll"])
    log(f"  ll={ll:.12g} oracle={rec['ll']:.12g} rel={rel:.2e} metric gate 1e-6: "
        f"{'met' if rel <= 1e-6 else 'NOT met'}; rank mean {i.rank_sum / max(1, 71 * 72 // 2 - i.dense_tiles):.1f} "
        f"max {i.rank_max} dense {i.dense_tiles}")
    h.close()
    with open(os.path.join(HERE, "golden", f"n40000_tlr_{eps:.0e}".replace("e-0", "e-") + ".json")) as f:
        otl = [r for r in json.load(f)["loglik"] if tuple(r["theta"]) == th][0]
    e_or = abs(otl["ll"] - rec["ll"]) / abs(rec["ll"])
    log(f"  oracle TLR at eps: rel {e_or:.2e} (rank mean {otl['rank_mean']:.1f})")
    assert rel <= max(10 * eps, 2.0 * e_or)


def _scores():
    with open(GOLD) as f:
        return json.load(f)["score"]


@pytest.mark.parametrize("rec", _scores(), ids=lambda r: f"s{r['theta'][0]}-b{r['theta'][1]}")
@pytest.mark.parametrize("mode", ["dense", "tlr"])
def test_score_n40000(rec, mode):
    import paper_1804_09137_amd as P
    th = tuple(rec["theta"])
    eps = 1e-7
    xd, yd, zd = _dev()
    log(f"score n=40000 {mode} theta={th}")
    h = P.Handle(40000, NB, mode=mode, tol=eps, want_grad=True)
    ll, (gs, gb) = h.loglik_grad(xd, yd, zd, th)
    h.close()
    scale = 0.5 * (abs(rec["tr_beta"]) + abs(rec["qf_beta"]))
    log(f"  ll={ll:.12g} vs {rec['ll']:.12g}; dsigma2 {gs:.10g} vs {rec['dsigma2']:.10g}; "
        f"dbeta {gb:.10g} vs {rec['dbeta']:.10g} (scale {scale:.3e})")
    if mode == "dense":
        assert abs(ll - rec["ll"]) <= 1e-9 * abs(rec["ll"])
        assert abs(gs - rec["dsigma2"]) <= 1e-8 * 0.5 * 40000 / th[0]
        assert abs(gb - rec["dbeta"]) <= 1e-8 * scale
    else:
        assert abs(ll - rec["ll"]) <= 10 * eps * abs(rec["ll"])
        assert abs(gs - rec["dsigma2"]) <= 100 * eps * 0.5 * 40000 / th[0]
        assert abs(gb - rec["dbeta"]) <= 100 * eps * scale


def test_central_difference_n40000():
    # dl/dbeta of the TLR score against a central difference of the dense
    # log-likelihood at h = 1e-6 (relative), at theta_true
    import paper_1804_09137_amd as P
    g, _, _, _ = _case()
    th = tuple(g["theta_true"])
    xd, yd, zd = _dev()
    d = P.Handle(40000, NB, mode="dense")
    hb = 1e-6 * th[1]
    vals = []
    for b in (th[1] + hb, th[1] - hb):
        d.generate(xd, yd, (th[0], b, th[2]))
        d.potrf()
        vals.append(d.loglik(zd)[0])
    d.close()
    fd = (vals[0] - vals[1]) / (2 * hb)
    t = P.Handle(40000, NB, tol=1e-7, want_grad=True)
    _, (_, gb) = t.loglik_grad(xd, yd, zd, th)
    t.close()
    ref = [r for r in g["score"] if tuple(r["theta"]) == th][0]
    scale = 0.5 * (abs(ref["tr_beta"]) + abs(ref["qf_beta"]))
    log(f"FD dl/dbeta {fd:.8g}, TLR score {gb:.8g}, oracle {ref['dbeta']:.8g}")
    # the difference quotient's rounding: ~1e-12 |l| / h
    assert abs(fd - gb) <= 1e-6 * scale + 4e-12 * abs(ref["ll"]) / hb


def test_lbfgs_mle_n40000():
    # L-BFGS from (0.5, 0.05) on the TLR likelihood and score (eps = 1e-7,
    # nu = 0.5 fixed) to a relative gradient tolerance of 1e-6; the result is
    # a maximum: the score vanishes there against the oracle's score scale at
    # theta_true, the likelihood is no lower than at theta_true, and a
    # derivative-free Nelder-Mead search on the same likelihood finds the same
    # point with more evaluations
    import paper_1804_09137_amd as P
    from paper_1804_09137_amd.autograd import fit
    g, _, _, _ = _case()
    nu = g["theta_true"][2]
    xd, yd, zd = _dev()
    h = P.Handle(40000, NB, tol=1e-7, want_grad=True)
    a = fit(h, xd, yd, zd, (0.5, 0.05), nu, tol=1e-6)
    ll_true = [r for r in g["loglik"] if tuple(r["theta"]) == tuple(g["theta_true"])][0]["ll"]
    ref = [r for r in g["score"] if tuple(r["theta"]) == tuple(g["theta_true"])][0]
    log(f"L-BFGS: theta {a['theta']} ll {a['ll']:.10g} score {a['grad']} in {a['evals']} evals "
        f"({a['message']}); ll(theta_true) {ll_true:.10g}")
    assert a["converged"]
    assert a["ll"] >= ll_true - 10 * 1e-7 * abs(ll_true)
    scale_b = 0.5 * (abs(ref["tr_beta"]) + abs(ref["qf_beta"]))
    assert abs(a["grad"][0]) <= 1e-5 * 0.5 * g["n"] / a["theta"][0]
    assert abs(a["grad"][1]) <= 1e-5 * scale_b
    b = fit(h, xd, yd, zd, (0.5, 0.05), nu, method="Nelder-Mead", tol=1e-6)
    h.close()
    log(f"Nelder-Mead: theta {b['theta']} ll {b['ll']:.10g} in {b['evals']} evals")
    np.testing.assert_allclose(a["theta"], b["theta"], rtol=1e-4)
    assert a["evals"] < b["evals"]
