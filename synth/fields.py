"""Seeded location grids, Gaussian draws and batched-field specifications.

Every generator uses numpy's PCG64 (``numpy.random.default_rng(seed)``); the
draw order is part of the contract and is stated in each docstring.
"""
from __future__ import annotations

from dataclasses import dataclass
import math

import numpy as np


def jittered_grid(m: int, seed: int = 0) -> tuple[np.ndarray, np.ndarray]:
    """Jittered m x m grid in the unit square (paper, Section VII).

    Draw order: X (m, m) then Y (m, m), both U(-0.4, 0.4) from
    ``default_rng(seed)``.  Point index p = (r - 1) * m + (l - 1) for
    r, l in 1..m (r-major); x_p = (r - 0.5 + X[r-1, l-1]) / m and
    y_p = (l - 0.5 + Y[r-1, l-1]) / m.

    Returns float64 arrays x, y of length m*m in generation order (unsorted).
    """
    if m < 1:
        raise ValueError("m must be >= 1")
    rng = np.random.default_rng(seed)
    X = rng.uniform(-0.4, 0.4, size=(m, m))
    Y = rng.uniform(-0.4, 0.4, size=(m, m))
    r = np.arange(1, m + 1, dtype=np.float64)[:, None]
    l = np.arange(1, m + 1, dtype=np.float64)[None, :]
    x = ((r - 0.5 + X) / m).reshape(-1)
    y = ((l - 0.5 + Y) / m).reshape(-1)
    return np.ascontiguousarray(x), np.ascontiguousarray(y)


def jittered_subset(n: int, seed: int = 0) -> tuple[np.ndarray, np.ndarray]:
    """n points of a ceil(sqrt(n))^2 jittered grid.

    The grid is ``jittered_grid(m, seed)``; when m*m > n a subset of n grid
    points is kept, chosen by ``default_rng(seed + 7919).choice(m*m, n,
    replace=False)`` and then sorted by grid index, so the result is in
    generation order.  When n is a perfect square the full grid is returned.
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    m = int(math.isqrt(n))
    if m * m < n:
        m += 1
    x, y = jittered_grid(m, seed)
    if m * m == n:
        return x, y
    keep = np.sort(np.random.default_rng(seed + 7919).choice(m * m, n, replace=False))
    return np.ascontiguousarray(x[keep]), np.ascontiguousarray(y[keep])


def standard_normal(n: int, seed: int = 1) -> np.ndarray:
    """n iid N(0, 1) draws from ``default_rng(seed).standard_normal(n)``."""
    return np.random.default_rng(seed).standard_normal(n)


@dataclass(frozen=True)
class FieldSpec:
    n: int
    sigma2: float
    beta: float
    nu: float
    loc_seed: int
    z_seed: int


def batched_field_specs(nfields: int = 64, seed: int = 0, n_lo: int = 2000,
                        n_hi: int = 20000) -> list[FieldSpec]:
    """Specifications of independent fields of uneven size.

    Draw order from ``default_rng(seed)``: n (integers in [n_lo, n_hi]),
    sigma2 ~ U(0.5, 2), beta ~ U(0.03, 0.3), then nu chosen from {0.5, 1.5};
    each array has length ``nfields``.  Field f uses location seed
    ``1000 + f`` and measurement seed ``2000 + f``.
    """
    rng = np.random.default_rng(seed)
    ns = rng.integers(n_lo, n_hi, size=nfields, endpoint=True)
    s2 = rng.uniform(0.5, 2.0, size=nfields)
    be = rng.uniform(0.03, 0.3, size=nfields)
    nu = rng.choice(np.array([0.5, 1.5]), size=nfields)
    return [FieldSpec(int(ns[f]), float(s2[f]), float(be[f]), float(nu[f]),
                      1000 + f, 2000 + f) for f in range(nfields)]
