"""Tile storage sized by the ranks (Section V: TLR memory follows sum nb k_ij).

* a factor takes U and V at each tile's own rank: the storage it reports is
  exactly sum over low-rank tiles of 2 nb k (rounded up per block) plus nb^2
  per dense tile, for both families with the gradient;
* a fixed budget (tlr_opts.arena_bytes) that is too small fails with
  TLR_ENOMEM and leaves the handle usable; the same budget raised to what the
  factor needs gives the same log-likelihood;
* automatic storage that starts too small is doubled and the pass redone,
  with an unchanged result.
"""
import os

import numpy as np
import pytest

from oracle import dense as D

from gpu_util import field, log, to_dev

pytestmark = pytest.mark.gpu


def _pad16(v):
    return (v + 15) // 16 * 16


def test_storage_follows_ranks():
    import paper_1804_09137_amd as P
    n, nb, eps = 3000, 256, 1e-8
    th = (1.0, 0.1, 0.5)
    x, y, z = field(n, 11, th)
    xd, yd, zd = to_dev(x, y, z)
    h = P.Handle(n, nb, tol=eps)
    h.generate(xd, yd, th)
    h.potrf()
    r = h.ranks()
    i = h.info()
    nt = h.nt
    want = 0
    for a in range(nt):
        for b in range(a):
            k = int(r[a, b])
            if k <= 0:
                continue
            want += _pad16(nb * k) if k >= nb or k > i.maxrank else 2 * _pad16(nb * k)
    log(f"tile storage {i.tile_bytes_used} B (cap {i.tile_bytes_cap}), from the ranks {8 * want} B; "
        f"dense {i.dense_tiles}; device {i.device_bytes / 2**20:.1f} MiB")
    assert i.tile_bytes_used == 8 * want
    assert i.tile_bytes_used <= i.tile_bytes_cap


def test_fixed_budget_too_small_is_enomem():
    import paper_1804_09137_amd as P
    n, nb, eps = 2000, 256, 1e-9
    th = (1.0, 0.1, 1.0)
    x, y, z = field(n, 12, th)
    xd, yd, zd = to_dev(x, y, z)
    ref = P.Handle(n, nb, tol=eps)
    ref.generate(xd, yd, th)
    ref.potrf()
    ll_ref, _, _ = ref.loglik(zd)
    need = ref.info().tile_bytes_used
    small = P.Handle(n, nb, tol=eps, arena_bytes=need // 4)
    small.generate(xd, yd, th)
    for _ in range(2):   # repeatable, and the handle survives it
        with pytest.raises(P.TLRError) as e:
            small.potrf()
        assert e.value.status == -2   # TLR_ENOMEM
    with pytest.raises(P.TLRError):
        small.loglik(zd)              # no factor: TLR_ESTATE
    ok = P.Handle(n, nb, tol=eps, arena_bytes=need)
    ok.generate(xd, yd, th)
    ok.potrf()
    ll, _, _ = ok.loglik(zd)
    log(f"need {need} B; ll {ll} vs {ll_ref}")
    assert ll == ll_ref
    assert ok.info().tile_bytes_cap == need


@pytest.mark.parametrize("grad", [False, True])
def test_automatic_storage_doubles(grad, monkeypatch):
    import paper_1804_09137_amd as P
    n, nb, eps = 2500, 256, 1e-9
    th = (1.0, 0.1, 0.5)
    x, y, z = field(n, 13, th)
    xd, yd, zd = to_dev(x, y, z)
    ref = D.gradient(x, y, z, th) if grad else D.loglik(x, y, z, th)
    out = []
    for start in (None, "20000"):
        if start:
            monkeypatch.setenv("TLR_ARENA_START", start)
        else:
            monkeypatch.delenv("TLR_ARENA_START", raising=False)
        h = P.Handle(n, nb, tol=eps, want_grad=grad)
        if grad:
            ll, g = h.loglik_grad(xd, yd, zd, th)
        else:
            h.generate(xd, yd, th)
            h.potrf()
            ll, _, _ = h.loglik(zd)
            g = None
        i = h.info()
        log(f"start {start}: grows {i.arena_grows} cap {i.tile_bytes_cap} used {i.tile_bytes_used} ll {ll}")
        out.append((ll, g, i.arena_grows))
        h.close()
    monkeypatch.delenv("TLR_ARENA_START", raising=False)
    # the default start may itself have been doubled (dense tiles beyond two
    # per tile column); the tiny start needs several doublings more
    assert out[1][2] >= out[0][2] + 3
    assert abs(out[1][0] - ref["ll"]) <= 10 * eps * abs(ref["ll"])
    # same sketches, same ranks: the redone pass gives the same result
    assert out[1][0] == out[0][0]
