"""Pins for oracle.ordering: brute-force bit interleaving and Z-curve shape."""
import numpy as np

from oracle import ordering as O


def _brute_key(qx, qy):
    bx = format(qx, "016b")
    by = format(qy, "016b")
    s = "".join(b + a for a, b in zip(bx, by))  # y bit above x bit, msb first
    return int(s, 2)


def test_keys_match_bit_string_interleave():
    rng = np.random.default_rng(5)
    x = rng.uniform(0, 1, 200)
    y = rng.uniform(0, 1, 200)
    keys = O.morton_keys(x, y)
    qx = np.floor(((x - x.min()) / (x.max() - x.min())) * 65535).astype(int)
    qy = np.floor(((y - y.min()) / (y.max() - y.min())) * 65535).astype(int)
    for i in range(200):
        assert keys[i] == _brute_key(int(qx[i]), int(qy[i]))


def test_quadrant_z_shape():
    # 2x2 grid: Z-curve visits (lo,lo), (hi,lo), (lo,hi), (hi,hi)
    x = np.array([1.0, 0.0, 1.0, 0.0])
    y = np.array([1.0, 1.0, 0.0, 0.0])
    p = O.morton_order(x, y)
    assert list(zip(x[p], y[p])) == [(0, 0), (1, 0), (0, 1), (1, 1)]


def test_stable_ties_and_degenerate_axis():
    x = np.array([0.5, 0.5, 0.5, 0.5])
    y = np.array([0.2, 0.1, 0.2, 0.1])
    p = O.morton_order(x, y)
    assert list(p) == [1, 3, 0, 2]


def test_is_permutation():
    rng = np.random.default_rng(1)
    x, y = rng.uniform(size=1000), rng.uniform(size=1000)
    p = O.morton_order(x, y)
    assert sorted(p.tolist()) == list(range(1000))
