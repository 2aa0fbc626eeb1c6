"""Shared fixtures of the GPU tests: seeded fields, ordered by the library's
own Morton helper, measurements drawn by the oracle."""
from __future__ import annotations

import functools
import sys

import numpy as np

import synth
from oracle import dense as D


def log(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


@functools.lru_cache(maxsize=16)
def field(n: int, seed: int = 0, theta=(1.0, 0.1, 0.5), with_z: bool = True):
    """(x, y, z) numpy arrays: jittered field of n points in Morton order, z = L eps."""
    from paper_1804_09137_amd import morton_order
    x, y = synth.jittered_subset(n, seed)
    p = morton_order(x, y)
    x, y = x[p].copy(), y[p].copy()
    z = D.sample_z(x, y, theta, synth.standard_normal(n, seed + 1)) if with_z else None
    return x, y, z


def to_dev(*arrs):
    import torch
    return tuple(torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda") for a in arrs)
