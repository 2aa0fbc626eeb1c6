"""MI355X-native tile low-rank (TLR) Matérn log-likelihood (arXiv 1804.09137).

Thin Python layer over the C-ABI of libtlrmle.so (include/tlr.h).  Every
step of the likelihood and its gradient runs in the library's HIP kernels;
this module only marshals torch device tensors, host scalars and status codes.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib

__all__ = ["TLRError", "NotSPDError", "RankError", "Handle", "morton_order", "loglik_grad_batched", "TLRLogLik"]


class TLRError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        detail = ""
        if status in (_lib.TLR_EHIP, _lib.TLR_ENOMEM):
            detail = " [" + _lib.load().tlr_last_error().decode(errors="replace") + "]"
        super().__init__(f"{what}: {_lib.status_name(status)}{detail}")
        self.status = status


class NotSPDError(TLRError):
    def __init__(self, info: int, what: str = ""):
        super().__init__(_lib.TLR_ENOTSPD, what)
        self.info = int(info)


class RankError(TLRError):
    def __init__(self, tile, what: str = ""):
        super().__init__(_lib.TLR_ERANK, what)
        self.tile = tile


def _check_len(t, count: int, what: str = "tensor"):
    """The C-ABI takes bare device pointers: a tensor shorter than the count
    the call reads or writes would be accessed out of bounds on the GPU."""
    if t.numel() < count:
        raise ValueError(f"{what}: expected at least {count} elements, got {t.numel()}")


def _ptr(t, count: int = None, what: str = "tensor") -> ctypes.c_void_p:
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError("expected a contiguous float64 torch tensor on the GPU")
    if count is not None:
        _check_len(t, count, what)
    return ctypes.c_void_p(t.data_ptr())


def _d3(v) -> ctypes.Array:
    a = (ctypes.c_double * 3)()
    for i in range(3):
        a[i] = float(v[i])
    return a


class Handle:
    """One problem size n on the current GPU.  mode: 'tlr' or 'dense'."""

    def __init__(self, n: int, nb: int, tol: float = 1e-9, maxrank: int = 0, mode: str = "tlr",
                 prec: str = "fp64", want_grad: bool = False, seed: int = 0, strict_rank: bool = False,
                 stream=None, single_stream: bool = False, arena_bytes: int = 0, metric: str = "euclid",
                 sphere_radius: float = 0.0, aca: bool = False, pivoted_trunc: bool = False):
        import torch
        self._lib = _lib.load()
        o = _lib.Opts()
        o.n, o.nb, o.maxrank, o.tol = int(n), int(nb), int(maxrank), float(tol)
        o.mode = {"tlr": _lib.MODE_TLR, "dense": _lib.MODE_DENSE}[mode]
        o.prec = {"fp64": _lib.PREC_FP64, "fp32_updates": _lib.PREC_FP32_UPDATES}[prec]
        o.want_grad = 1 if want_grad else 0
        o.seed = int(seed)
        o.flags = ((_lib.FLAG_STRICT_RANK if strict_rank else 0) | (_lib.FLAG_SINGLE_STREAM if single_stream else 0)
                   | (_lib.FLAG_ACA if aca else 0) | (_lib.FLAG_PIVOTED_TRUNC if pivoted_trunc else 0))
        o.arena_bytes = int(arena_bytes)
        o.metric = {"euclid": 0, "great_circle": 1}[metric]
        o.sphere_radius = float(sphere_radius)
        self.n, self.nb, self.mode = int(n), int(nb), mode
        self.nt = (self.n + self.nb - 1) // self.nb
        if stream is None:
            stream = torch.cuda.current_stream()
        self._stream = stream
        self._h = ctypes.c_void_p()
        st = self._lib.tlr_create(ctypes.byref(self._h), ctypes.byref(o), ctypes.c_void_p(stream.cuda_stream))
        if st != _lib.TLR_OK:
            raise TLRError(st, "tlr_create")
        self._keep = ()

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.tlr_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int, what: str, info: int = 0):
        if st == _lib.TLR_OK:
            return
        if st == _lib.TLR_ENOTSPD:
            raise NotSPDError(info, what)
        if st == _lib.TLR_ERANK:
            i = self.info()
            raise RankError((i.bad_tile_i, i.bad_tile_j), what)
        raise TLRError(st, what)

    def generate(self, x, y, theta):
        st = self._lib.tlr_generate(self._h, _ptr(x, self.n, "x"), _ptr(y, self.n, "y"), _d3(theta))
        self._check(st, "tlr_generate")
        self._keep = (x, y)

    def compress(self):
        self._check(self._lib.tlr_compress(self._h), "tlr_compress")

    def potrf(self) -> int:
        info = ctypes.c_int64(0)
        st = self._lib.tlr_potrf(self._h, ctypes.byref(info))
        self._check(st, "tlr_potrf", info.value)
        return info.value

    def loglik(self, z):
        ll, ld, q = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        st = self._lib.tlr_loglik(self._h, _ptr(z, self.n, "z"), ctypes.byref(ll), ctypes.byref(ld), ctypes.byref(q))
        self._check(st, "tlr_loglik")
        return ll.value, ld.value, q.value

    def loglik_grad(self, x, y, z, theta):
        ll = ctypes.c_double()
        g = (ctypes.c_double * 2)()
        info = ctypes.c_int64(0)
        st = self._lib.tlr_loglik_grad(self._h, _ptr(x, self.n, "x"), _ptr(y, self.n, "y"), _ptr(z, self.n, "z"),
                                       _d3(theta), ctypes.byref(ll), g, ctypes.byref(info))
        self._check(st, "tlr_loglik_grad", info.value)
        self._keep = (x, y)
        return ll.value, (g[0], g[1])

    def predict(self, z, xnew, ynew, variance: bool = False):
        """Kriging prediction at (xnew, ynew) from the observed z (after
        potrf): Sigma_12 Sigma_22^{-1} z, and the conditional variances if
        asked (Section III)."""
        import torch
        m = int(xnew.shape[0])
        pred = torch.empty(m, dtype=torch.float64, device="cuda")
        var = torch.empty(m, dtype=torch.float64, device="cuda") if variance else None
        st = self._lib.tlr_predict(self._h, _ptr(z, self.n, "z"), m, _ptr(xnew), _ptr(ynew, m, "ynew"), _ptr(pred),
                                   _ptr(var) if variance else ctypes.c_void_p())
        self._check(st, "tlr_predict")
        return (pred, var) if variance else pred

    def loglik_grad3(self, x, y, z, theta):
        """l and (dl/dsigma^2, dl/dbeta, dl/dnu) (tlr_loglik_grad3)."""
        ll = ctypes.c_double()
        g = (ctypes.c_double * 3)()
        info = ctypes.c_int64(0)
        st = self._lib.tlr_loglik_grad3(self._h, _ptr(x, self.n, "x"), _ptr(y, self.n, "y"), _ptr(z, self.n, "z"),
                                        _d3(theta), ctypes.byref(ll), g, ctypes.byref(info))
        self._check(st, "tlr_loglik_grad3", info.value)
        self._keep = (x, y)
        return ll.value, (g[0], g[1], g[2])

    def sample(self, eps):
        """z = L eps with the current factor (after potrf)."""
        import torch
        z = torch.empty_like(eps)
        self._check(self._lib.tlr_sample(self._h, _ptr(eps, self.n, "eps"), _ptr(z)), "tlr_sample")
        return z

    def profile(self, enable=True):
        """Per-kernel-class hipEvent timing (resets the counters): False/0 off,
        True/1 on, 2 on with every column-update group run alone so that its
        events time only its own kernels."""
        mode = 2 if enable == 2 else (1 if enable else 0)
        self._check(self._lib.tlr_profile(self._h, mode), "tlr_profile")

    def kstats(self) -> dict:
        arr = (_lib.KStat * len(_lib.KCLASSES))()
        self._check(self._lib.tlr_get_kstats(self._h, arr), "tlr_get_kstats")
        return {name: {"launches": a.launches, "ms": a.ms, "flops": a.flops, "bytes": a.bytes}
                for name, a in zip(_lib.KCLASSES, arr)}

    def ranks(self) -> np.ndarray:
        out = np.zeros(self.nt * self.nt, dtype=np.int32)
        st = self._lib.tlr_get_ranks(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
        self._check(st, "tlr_get_ranks")
        return out.reshape(self.nt, self.nt)

    def tangent_ranks(self) -> np.ndarray:
        """Ranks of the tangent factor's tiles after loglik_grad (TLR)."""
        out = np.zeros(self.nt * self.nt, dtype=np.int32)
        st = self._lib.tlr_get_tangent_ranks(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
        self._check(st, "tlr_get_tangent_ranks")
        return out.reshape(self.nt, self.nt)

    def info(self) -> _lib.Info:
        i = _lib.Info()
        self._lib.tlr_get_info(self._h, ctypes.byref(i))
        return i

    def tile(self, i: int, j: int):
        import torch
        mi = min(self.nb, self.n - i * self.nb)
        mj = min(self.nb, self.n - j * self.nb)
        out = torch.empty((mj, mi), dtype=torch.float64, device="cuda")   # column-major mi x mj
        st = self._lib.tlr_get_tile(self._h, int(i), int(j), _ptr(out), mi)
        self._check(st, "tlr_get_tile")
        return out.t()

    def covariance_block(self, r0: int, m: int, c0: int, k: int, deriv=False):
        """Sigma block (deriv False/0), dSigma/dbeta (True/1 or "beta") or dSigma/dnu (2 or "nu")."""
        import torch
        out = torch.empty((k, m), dtype=torch.float64, device="cuda")
        dv = {"beta": 1, "nu": 2}[deriv] if isinstance(deriv, str) else int(deriv)
        st = self._lib.tlr_covariance_block(self._h, int(r0), int(m), int(c0), int(k), dv,
                                            _ptr(out), int(m))
        self._check(st, "tlr_covariance_block")
        return out.t()


def loglik_grad_batched(handles, xs, ys, zs, thetas, nthreads: int = 4):
    """l and dl/d(sigma^2, beta) of several independent fields, one Handle
    each (built with want_grad=True, on distinct streams), evaluated
    concurrently by tlr_loglik_grad_batched.  Returns (ll[nf], grad[nf, 2]);
    raises the first failing field's error."""
    nf = len(handles)
    if not (len(xs) == len(ys) == len(zs) == len(thetas) == nf):
        raise ValueError("one x, y, z and theta per handle")
    lib = _lib.load()
    P = ctypes.c_void_p
    hs = (P * nf)(*[h._h.value for h in handles])
    px = (P * nf)(*[_ptr(t, h.n, f"x[{f}]").value for f, (h, t) in enumerate(zip(handles, xs))])
    py = (P * nf)(*[_ptr(t, h.n, f"y[{f}]").value for f, (h, t) in enumerate(zip(handles, ys))])
    pz = (P * nf)(*[_ptr(t, h.n, f"z[{f}]").value for f, (h, t) in enumerate(zip(handles, zs))])
    th = np.ascontiguousarray(np.asarray(thetas, dtype=np.float64).reshape(nf, 3))
    ll = np.zeros(nf)
    gr = np.zeros((nf, 2))
    info = np.zeros(nf, dtype=np.int64)
    st = np.zeros(nf, dtype=np.int32)
    dp = ctypes.POINTER(ctypes.c_double)
    rc = lib.tlr_loglik_grad_batched(nf, hs, px, py, pz, th.ctypes.data_as(dp), ll.ctypes.data_as(dp),
                                     gr.ctypes.data_as(dp), info.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                     st.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), int(nthreads))
    if rc != _lib.TLR_OK:
        f = int(np.flatnonzero(st != _lib.TLR_OK)[0]) if np.any(st != _lib.TLR_OK) else 0
        handles[f]._check(int(st[f]) if np.any(st != _lib.TLR_OK) else rc, f"tlr_loglik_grad_batched field {f}",
                          int(info[f]))
    for h, x, y in zip(handles, xs, ys):
        h._keep = (x, y)
    return ll, gr


def dense_loglik_noalloc(x, y, z, theta, stream=None):
    """Dense l, log|Sigma| and z^T Sigma^{-1} z of one small field (n <= 2048)
    with no handle and no device allocation (tlr_dense_loglik_noalloc)."""
    import torch
    lib = _lib.load()
    n = int(x.shape[0])
    ll, ld, q = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    info = ctypes.c_int64(0)
    s = stream if stream is not None else torch.cuda.current_stream()
    st = lib.tlr_dense_loglik_noalloc(n, _ptr(x), _ptr(y, n, "y"), _ptr(z, n, "z"), _d3(theta), ctypes.byref(ll), ctypes.byref(ld),
                                      ctypes.byref(q), ctypes.byref(info), ctypes.c_void_p(s.cuda_stream))
    if st == _lib.TLR_ENOTSPD:
        raise NotSPDError(info.value, "tlr_dense_loglik_noalloc")
    if st != _lib.TLR_OK:
        raise TLRError(st, "tlr_dense_loglik_noalloc")
    return ll.value, ld.value, q.value


def morton_order(x, y) -> np.ndarray:
    """Host Morton (Z-order) permutation of the points (x[i], y[i])."""
    lib = _lib.load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    n = x.shape[0]
    perm = np.empty(n, dtype=np.int64)
    dp = ctypes.POINTER(ctypes.c_double)
    st = lib.tlr_morton_order(n, x.ctypes.data_as(dp), y.ctypes.data_as(dp),
                              perm.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    if st != _lib.TLR_OK:
        raise TLRError(st, "tlr_morton_order")
    return perm


def __getattr__(name):
    if name == "TLRLogLik":
        from .autograd import TLRLogLik
        return TLRLogLik
    raise AttributeError(name)
