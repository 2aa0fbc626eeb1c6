"""Morton (Z-order) ordering of 2-D locations.

The paper never states a point ordering, yet the ranks of the off-diagonal
tiles depend on it.  Reading adopted by the build: quantise each coordinate to
16 bits over the bounding box of the points,
    q = floor(((c - cmin) / (cmax - cmin)) * 65535)
(q = 0 for every point when cmax == cmin), interleave the bits with x on the
even positions and y on the odd positions, and sort the 32-bit keys stably
(ties keep their input order).
"""
from __future__ import annotations

import numpy as np


def _quantise(c: np.ndarray) -> np.ndarray:
    c = np.asarray(c, dtype=np.float64)
    lo = c.min()
    w = c.max() - lo
    if w == 0.0:
        return np.zeros(c.shape, dtype=np.int64)
    return np.floor(((c - lo) / w) * 65535.0).astype(np.int64)


def morton_keys(x, y) -> np.ndarray:
    """32-bit Morton keys, bit b of qx -> bit 2b, bit b of qy -> bit 2b+1."""
    qx = _quantise(x)
    qy = _quantise(y)
    key = np.zeros(qx.shape, dtype=np.int64)
    for b in range(16):
        key |= ((qx >> b) & 1) << (2 * b)
        key |= ((qy >> b) & 1) << (2 * b + 1)
    return key


def morton_order(x, y) -> np.ndarray:
    """Permutation p (int64) such that points p[0], p[1], ... follow the Z-curve."""
    return np.argsort(morton_keys(x, y), kind="stable").astype(np.int64)
