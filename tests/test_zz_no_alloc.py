"""The allocation-free dense log-likelihood entry point against the existing
dense entry points (tlr_create DENSE + tlr_generate + tlr_potrf +
tlr_loglik), through the C-ABI: two calls in a row, the second with a smaller
field (the shared device array keeps the first call's contents), plus its
size limit and the not-positive-definite report."""
import ctypes

import numpy as np
import pytest

from gpu_util import field, log, to_dev

pytestmark = pytest.mark.gpu


def _noalloc(lib, n, xd, yd, zd, th):
    import torch
    ll, ld, q = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    info = ctypes.c_int64(0)
    t3 = (ctypes.c_double * 3)(*th)
    st = lib.tlr_dense_loglik_noalloc(n, ctypes.c_void_p(xd.data_ptr()), ctypes.c_void_p(yd.data_ptr()),
                                      ctypes.c_void_p(zd.data_ptr()), t3, ctypes.byref(ll), ctypes.byref(ld),
                                      ctypes.byref(q), ctypes.byref(info),
                                      ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st, ll.value, ld.value, q.value, info.value


def _lib():
    from paper_1804_09137_amd import _lib as L
    lib = L.load()
    P = ctypes.c_void_p
    D = ctypes.POINTER(ctypes.c_double)
    lib.tlr_dense_loglik_noalloc.argtypes = [ctypes.c_int64, P, P, P, D, D, D, D, ctypes.POINTER(ctypes.c_int64), P]
    lib.tlr_dense_loglik_noalloc.restype = ctypes.c_int
    return lib


def test_noalloc_matches_dense_entry_points_twice():
    import paper_1804_09137_amd as P
    lib = _lib()
    for n, th in ((2000, (1.0, 0.1, 0.5)), (777, (1.3, 0.07, 1.0))):
        x, y, z = field(n, 81, th)
        xd, yd, zd = to_dev(x, y, z)
        st, ll, ld, q, info = _noalloc(lib, n, xd, yd, zd, th)
        assert st == 0, st
        h = P.Handle(n, 256, mode="dense")
        h.generate(xd, yd, th)
        h.potrf()
        ll2, ld2, q2 = h.loglik(zd)
        h.close()
        log(f"n={n}: noalloc ll {ll!r}, dense handle {ll2!r}")
        assert abs(ll - ll2) <= 1e-12 * abs(ll2)
        assert abs(ld - ld2) <= 1e-12 * abs(ld2)
        assert abs(q - q2) <= 1e-12 * abs(q2)


def test_noalloc_limits_and_not_spd():
    import torch
    lib = _lib()
    x, y, z = field(300, 82, (1.0, 0.1, 0.5))
    xd, yd, zd = to_dev(x, y, z)
    big = torch.zeros(2049, dtype=torch.float64, device="cuda")
    st, *_ = _noalloc(lib, 2049, big, big, big, (1.0, 0.1, 0.5))
    assert st == -1
    assert b"exceeds the maximum 2048" in lib.tlr_last_error()
    st, *_, info = _noalloc(lib, 300, xd, yd, zd, (-1.0, 0.1, 0.5))
    assert st == 1 and info == 1
    st, ll, *_ = _noalloc(lib, 300, xd, yd, zd, (1.0, 0.1, 0.5))
    assert st == 0 and np.isfinite(ll)
