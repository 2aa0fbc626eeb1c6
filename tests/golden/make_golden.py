"""Writes the stored expected values of the large parity tests.

Calls only the CPU oracle (``oracle/``) and the seeded input generators
(``synth``); nothing here touches the HIP library.  Run from the repository
root, e.g.

    python tests/golden/make_golden.py n40000

Each configuration writes ``tests/golden/<name>.json`` (the oracle's results)
and ``tests/golden/<name>_z.npy`` (the measurement vector the results refer to).

n40000: the 200 x 200 jittered grid (locations seed 0), Morton order, the
measurement z = L eps of the field at theta_true = (1, 0.1, 0.5) (eps seed 1,
Section VIII-D); log-likelihood Eq. (1) at the six theta = (1, beta, nu),
beta in {0.03, 0.1, 0.3}, nu in {0.5, 1.0}; the score in (sigma^2, beta) at
theta_true and at the optimiser's start (0.5, 0.05, 0.5).

n102400: the 320 x 320 grid, theta = (1, 0.1, 0.5): z = L eps, the
log-determinant and q = z^T Sigma^{-1} z from the same factor.

n40000_tlr EPS: the oracle's tile low-rank log-likelihood of the n40000
configurations at threshold EPS (``tests/golden/n40000_tlr_EPS.json``).
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import ordering as O  # noqa: E402
from oracle import tiled as T  # noqa: E402


def _field(m: int):
    x, y = synth.jittered_grid(m, 0)
    p = O.morton_order(x, y)
    return x[p].copy(), y[p].copy()


def _save_z(name: str, z: np.ndarray) -> str:
    path = os.path.join(HERE, f"{name}_z.npy")
    np.save(path, z)
    return hashlib.sha256(z.tobytes()).hexdigest()


def _log(msg: str):
    print(msg, flush=True)


def n40000(nb: int = 2000) -> dict:
    m, name = 200, "n40000"
    x, y = _field(m)
    n = x.shape[0]
    th_true = (1.0, 0.1, 0.5)
    t0 = time.time()
    z = T.sample_z(x, y, th_true, synth.standard_normal(n, 1), nb=nb)
    _log(f"z done {time.time() - t0:.0f}s")
    out = {"n": n, "grid": m, "loc_seed": 0, "eps_seed": 1, "order": "morton",
           "theta_true": list(th_true), "z_sha256": _save_z(name, z), "loglik": [], "score": []}
    for beta in (0.03, 0.1, 0.3):
        for nu in (0.5, 1.0):
            th = (1.0, beta, nu)
            t0 = time.time()
            try:
                r = T.loglik(x, y, z, th, nb=nb)
                rec = {"theta": list(th), "ll": r["ll"], "logdet": r["logdet"], "quad": r["quad"]}
            except ArithmeticError as e:  # NotSPDError: recorded, not skipped silently
                rec = {"theta": list(th), "not_spd": getattr(e, "info", -1)}
            rec["oracle_s"] = round(time.time() - t0, 1)
            out["loglik"].append(rec)
            _log(f"loglik {th} {rec}")
    for th in (th_true, (0.5, 0.05, 0.5)):
        t0 = time.time()
        g = T.gradient(x, y, z, th, nb=nb)
        rec = {"theta": list(th), **{k: float(v) for k, v in g.items()}, "oracle_s": round(time.time() - t0, 1)}
        out["score"].append(rec)
        _log(f"score {th} {rec}")
    return out


def n102400(nb: int = 2048) -> dict:
    m, name = 320, "n102400"
    x, y = _field(m)
    n = x.shape[0]
    th = (1.0, 0.1, 0.5)
    t0 = time.time()
    L = T.cholesky_tiles(T.covariance_tiles(x, y, th, nb))
    z = T.lower_matvec(L, synth.standard_normal(n, 1))
    logdet = 2.0 * sum(float(np.sum(np.log(np.diag(L.t[k][k])))) for k in range(L.nt))
    w = T.forward_solve(L, z)
    quad = float(w @ w)
    ll = T._ll(n, logdet, quad)
    _log(f"n102400 done {time.time() - t0:.0f}s ll={ll}")
    return {"n": n, "grid": m, "loc_seed": 0, "eps_seed": 1, "order": "morton", "theta_true": list(th),
            "z_sha256": _save_z(name, z),
            "loglik": [{"theta": list(th), "ll": ll, "logdet": logdet, "quad": quad,
                        "oracle_s": round(time.time() - t0, 1)}]}


def n40000_tlr(eps: float) -> dict:
    """The oracle's own tile low-rank log-likelihood (oracle/tlr.py: SVD
    compression at eps, right-looking TLR Cholesky with QR + SVD
    recompression, tile 560) at the six theta of n40000, on the same z: the
    error of an exact-truncation TLR approximation at eps, against which the
    GPU's TLR error is judged where it exceeds 10 eps (smooth, strongly
    correlated fields)."""
    from oracle import tlr as OT
    m = 200
    x, y = _field(m)
    z = np.load(os.path.join(HERE, "n40000_z.npy"))
    out = {"n": x.shape[0], "nb": 560, "eps": eps, "loglik": []}
    for beta in (0.03, 0.1, 0.3):
        for nu in (0.5, 1.0):
            th = (1.0, beta, nu)
            t0 = time.time()
            r = OT.loglik(x, y, z, th, 560, eps)
            rk = r["ranks_factor"]
            low = rk[np.tril_indices(rk.shape[0], -1)]
            rec = {"theta": list(th), "ll": r["ll"], "logdet": r["logdet"], "quad": r["quad"],
                   "rank_mean": float(low.mean()), "rank_max": int(low.max()), "oracle_s": round(time.time() - t0, 1)}
            out["loglik"].append(rec)
            _log(f"tlr eps={eps} {th} {rec}")
    return out


if __name__ == "__main__":
    which = sys.argv[1]
    if which == "n40000_tlr":
        eps = float(sys.argv[2])
        res = n40000_tlr(eps)
        which = f"n40000_tlr_{sys.argv[2]}"
    else:
        res = {"n40000": n40000, "n102400": n102400}[which]()
    res["generator"] = "tests/golden/make_golden.py " + " ".join(sys.argv[1:])
    with open(os.path.join(HERE, f"{which}.json"), "w") as f:
        json.dump(res, f, indent=1)
    _log("written")
