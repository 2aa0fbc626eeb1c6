"""Algorithmic work of one TLR evaluation, from its rank tables.

These are the per-unit costs of the tile low-rank Cholesky of Section V
(the work the method must do, not the dense work it avoids), summed over the
ranks a factorisation actually produced.  Notation: tile (i, j) of rank
k_ij, tile sizes m_t (the last one ragged), p = k_ij + min(k_ik, k_jk) the
width of a recompression.

  a3 compression       per tile  4 m_i m_j (k_ij + 8) flops (randomized range
                                 finder with 8 extra samples, or QR with
                                 column pivoting), 8 m_i m_j + 16 nb k_ij bytes
                                 (read the tile once, write U and V)
  a4 POTRF             per column  m_k^3 / 3 flops, 16 m_k^2 bytes
  a5 TRSM              per tile  m_k^2 k_ik flops (V_ik <- L_kk^{-1} V_ik)
  a6 SYRK              per tile  4 m_i k_ik^2 + 2 m_i^2 k_ik flops
  a7 GEMM + recompression, per (i, j, k) with i > j > k:
                       4 nb k_ik k_jk + 4 nb p^2 + 4 nb p k_ij + 22 p^3 flops,
                       8 nb (2 k_ik + 2 k_jk + 4 k_ij) bytes
  a9 solve             8 (sum m_t^2 + sum 2 nb k_ij) bytes per sweep

A tile kept dense counts with its width as rank.  The tangent factor of the
gradient (forward mode, dL = derivative of the factor) repeats a3-a7 with two
products per update, dL_ik L_jk^T + L_ik dL_jk^T: both enter the product
term, and the recompression width is p = k'_ij + min(k'_ik, k_jk) +
min(k_ik, k'_jk) (k' the tangent's ranks).  The a3-a7 unit costs use the
final ranks as the ranks of every intermediate step.
"""
from __future__ import annotations

import numpy as np


def _sizes(n: int, nb: int) -> np.ndarray:
    nt = (n + nb - 1) // nb
    return np.array([min(nb, n - t * nb) for t in range(nt)], dtype=np.float64)


def factor_work(R: np.ndarray, n: int, nb: int, Rt: np.ndarray | None = None) -> dict:
    """Flops and bytes per row of the model above; R (and the tangent's Rt)
    are nt x nt rank tables, entries (i, j) for i > j used."""
    m = _sizes(n, nb)
    nt = m.shape[0]
    R = np.tril(np.asarray(R, dtype=np.float64), -1)
    out = {"compress": [0.0, 0.0], "potrf": [0.0, 0.0], "trsm": [0.0, 0.0], "syrk": [0.0, 0.0],
           "gemm_recompress": [0.0, 0.0], "solve": [0.0, 0.0]}

    def add(key, f, b):
        out[key][0] += float(f)
        out[key][1] += float(b)

    fams = [(R, None)] if Rt is None else [(R, None), (np.tril(np.asarray(Rt, dtype=np.float64), -1), R)]
    for F, P in fams:
        mi = m[:, None]
        mj = m[None, :]
        low = np.tril(np.ones((nt, nt)), -1)
        add("compress", np.sum(low * 4.0 * mi * mj * (F + 8.0)), np.sum(low * (8.0 * mi * mj + 16.0 * nb * F)))
        add("potrf", np.sum(m ** 3) / 3.0, 16.0 * np.sum(m ** 2))
        add("trsm", np.sum(low * (mj ** 2) * F), np.sum(low * 16.0 * nb * F))
        add("syrk", np.sum(low * (4.0 * mi * F ** 2 + 2.0 * mi ** 2 * F)), np.sum(low * 16.0 * nb * F))
        for k in range(nt - 2):
            a = F[k + 1:, k]                      # k_ik for i > k
            if P is None:
                prod = 4.0 * nb * np.outer(a, a)   # (i, j) -> 4 nb k_ik k_jk
                mn = np.minimum.outer(a, a)
                kij = F[k + 1:, k + 1:]
                p = kij + mn
                side = 2.0 * a[:, None] + 2.0 * a[None, :]
            else:
                b = P[k + 1:, k]                   # primal k_ik
                prod = 4.0 * nb * (np.outer(a, b) + np.outer(b, a))
                kij = F[k + 1:, k + 1:]
                p = kij + np.minimum.outer(a, b) + np.minimum.outer(b, a)
                side = 2.0 * (a + b)[:, None] + 2.0 * (a + b)[None, :]
            tri = np.tril(np.ones_like(kij), -1)   # i > j
            fl = prod + 4.0 * nb * p ** 2 + 4.0 * nb * p * kij + 22.0 * p ** 3
            add("gemm_recompress", np.sum(tri * fl), np.sum(tri * 8.0 * nb * (side + 4.0 * kij)))
        add("solve", 0.0, 8.0 * (np.sum(m ** 2) + np.sum(2.0 * nb * F)))
    tot_f = sum(v[0] for v in out.values())
    tot_b = sum(v[1] for v in out.values())
    res = {k: {"flops": v[0], "bytes": v[1]} for k, v in out.items()}
    res["total"] = {"flops": tot_f, "bytes": tot_b}
    return res


def rank_histogram(R: np.ndarray, edges=(0, 1, 4, 8, 16, 32, 64, 128, 256, 512, 1025)) -> dict:
    """Counts of strictly-lower tiles by rank, bins [edges[i], edges[i+1])."""
    R = np.asarray(R)
    low = R[np.tril_indices(R.shape[0], -1)]
    h, _ = np.histogram(low, bins=np.asarray(edges))
    return {f"{edges[i]}-{edges[i + 1] - 1}": int(h[i]) for i in range(len(h))}
