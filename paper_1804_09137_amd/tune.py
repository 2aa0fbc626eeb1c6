"""Autotuner of the tile size nb and the rank cap maxrank of a TLR handle.

The paper tunes its tile size per system and method (Section VIII-C: 560 for
the dense full-tile Cholesky, 1900 for TLR on Shaheen-2); the best tile here
depends on n, the threshold and the field's ranks.  The tuner times the
library itself: for each candidate (nb, maxrank) it builds a gradient handle,
runs one warm-up evaluation (which also gives the handle its rank history) and
then `reps` timed tlr_loglik_grad calls, and keeps the fastest.  Results are
cached per (n, eps, rounded theta) for the process.
"""
from __future__ import annotations

import time

_cache: dict = {}


def candidates(n: int, nbs=(400, 512, 640, 800, 1024), rank_fracs=(4, 3)) -> list[tuple[int, int]]:
    """(nb, maxrank) pairs worth timing for n points: tile sizes that are
    multiples of 16 in [32, 1024] and give at least 4 tile columns, each with
    maxrank = nb / f for the given fractions."""
    out = []
    for nb in nbs:
        if nb % 16 or not 32 <= nb <= 1024 or (n + nb - 1) // nb < 4:
            continue
        for f in rank_fracs:
            out.append((int(nb), int(nb // f)))
    if not out:   # small n: one tile size that still cuts the matrix in tiles
        nb = max(32, min(1024, (n // 4) // 16 * 16))
        out.append((nb, nb // 4))
    return out


def choose(timings: dict) -> tuple[int, int]:
    """The (nb, maxrank) of the smallest time (ties: the smaller nb)."""
    return min(timings, key=lambda k: (timings[k], k[0], k[1]))


def tune(x, y, z, theta, eps: float, cands=None, reps: int = 2, want_grad: bool = True, log=None) -> dict:
    """Time every candidate on (x, y, z, theta) and return {'nb', 'maxrank',
    'ms': {(nb, maxrank): ms per evaluation}}."""
    import torch
    from . import Handle
    n = int(x.shape[0])
    key = (n, float(eps), tuple(round(float(t), 3) for t in theta), bool(want_grad))
    if key in _cache:
        return _cache[key]
    cands = cands or candidates(n)
    ms = {}
    for nb, mr in cands:
        h = Handle(n, nb, tol=eps, maxrank=mr, want_grad=want_grad)
        try:
            run = (lambda: h.loglik_grad(x, y, z, theta)) if want_grad else (lambda: (h.generate(x, y, theta),
                                                                                     h.potrf()))
            run()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                run()
            torch.cuda.synchronize()
            ms[(nb, mr)] = 1e3 * (time.perf_counter() - t0) / reps
        finally:
            h.close()
            del h
            torch.cuda.empty_cache()
        if log:
            log(f"[tune] nb={nb} maxrank={mr}: {ms[(nb, mr)]:.1f} ms")
    nb, mr = choose(ms)
    res = {"nb": nb, "maxrank": mr, "ms": ms}
    _cache[key] = res
    return res
