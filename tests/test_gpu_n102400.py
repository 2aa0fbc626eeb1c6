"""GPU parity at the headline workload: n = 102,400 (320 x 320 jittered
grid, Morton order), theta = (1, 0.1, 0.5).  The expected log-likelihood is the
CPU oracle's (tiled dense Cholesky, ``tests/golden/n102400.json`` from
``tests/golden/make_golden.py n102400``), on the z = L eps stored beside it.

Dense FP64 (tile 512) within 1e-9 |l|; TLR (tile 800, the bench's
configuration) within 10 eps |l| at eps = 1e-7, which also meets the metric's
gate |dl| <= 1e-6 |l|.
"""
import hashlib
import json
import os

import numpy as np
import pytest

import synth

from gpu_util import log, to_dev

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def _case():
    import paper_1804_09137_amd as P
    with open(os.path.join(HERE, "golden", "n102400.json")) as f:
        g = json.load(f)
    x, y = synth.jittered_grid(g["grid"], g["loc_seed"])
    p = P.morton_order(x, y)
    x, y = x[p].copy(), y[p].copy()
    z = np.load(os.path.join(HERE, "golden", "n102400_z.npy"))
    assert hashlib.sha256(z.tobytes()).hexdigest() == g["z_sha256"]
    return g, x, y, z


@pytest.mark.parametrize("mode,nb,eps", [("dense", 512, 0.0), ("tlr", 800, 1e-7)])
def test_loglik_n102400(mode, nb, eps):
    import torch
    import paper_1804_09137_amd as P
    g, x, y, z = _case()
    rec = g["loglik"][0]
    th = tuple(rec["theta"])
    xd, yd, zd = to_dev(x, y, z)
    log(f"n=102400 {mode} nb={nb} eps={eps}")
    h = P.Handle(102400, nb, mode=mode, tol=max(eps, 1e-9), maxrank=256)
    h.generate(xd, yd, th)
    h.potrf()
    ll, ld, q = h.loglik(zd)
    h.close()
    del h
    torch.cuda.empty_cache()
    rel = abs(ll - rec["ll"]) / abs(rec["ll"])
    log(f"  ll={ll:.12g} oracle={rec['ll']:.12g} rel={rel:.2e}; logdet rel "
        f"{abs(ld - rec['logdet']) / abs(rec['logdet']):.2e}")
    if mode == "dense":
        assert rel <= 1e-9
        assert abs(ld - rec["logdet"]) <= 1e-9 * abs(rec["logdet"])
        assert abs(q - rec["quad"]) <= 1e-9 * abs(rec["quad"])
    else:
        assert rel <= 10 * eps
        assert rel <= 1e-6
