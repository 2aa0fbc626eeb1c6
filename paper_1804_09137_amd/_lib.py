"""ctypes binding of libtlrmle.so (the C-ABI declared in include/tlr.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Device buffers are torch CUDA (HIP) float64 tensors; the handle
enqueues on the torch stream that is current when the handle is created.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtlrmle.so")

TLR_OK = 0
TLR_ENOTSPD = 1
TLR_EINVAL = -1
TLR_ENOMEM = -2
TLR_EHIP = -3
TLR_ERANK = -4
TLR_ENOTIMPL = -5
TLR_ESTATE = -6

MODE_TLR = 0
MODE_DENSE = 1
PREC_FP64 = 0
PREC_FP32_UPDATES = 1
FLAG_STRICT_RANK = 1
FLAG_SINGLE_STREAM = 2
FLAG_ACA = 4
FLAG_PIVOTED_TRUNC = 8

_NAMES = {0: "TLR_OK", 1: "TLR_ENOTSPD", -1: "TLR_EINVAL", -2: "TLR_ENOMEM", -3: "TLR_EHIP",
          -4: "TLR_ERANK", -5: "TLR_ENOTIMPL", -6: "TLR_ESTATE"}


class Opts(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nb", ctypes.c_int32), ("maxrank", ctypes.c_int32),
                ("tol", ctypes.c_double), ("mode", ctypes.c_int32), ("prec", ctypes.c_int32),
                ("want_grad", ctypes.c_int32), ("seed", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("metric", ctypes.c_int32), ("arena_bytes", ctypes.c_int64), ("sphere_radius", ctypes.c_double)]


class Info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nb", ctypes.c_int32), ("nt", ctypes.c_int32),
                ("maxrank", ctypes.c_int32), ("mode", ctypes.c_int32), ("device_bytes", ctypes.c_int64),
                ("rank_sum", ctypes.c_int64), ("rank_max", ctypes.c_int32), ("dense_tiles", ctypes.c_int32),
                ("bad_tile_i", ctypes.c_int32), ("bad_tile_j", ctypes.c_int32),
                ("prec_used", ctypes.c_int32), ("fp64_retries", ctypes.c_int32), ("t_factor_ms", ctypes.c_double),
                ("t_solve_ms", ctypes.c_double), ("t_grad_ms", ctypes.c_double),
                ("tile_bytes_used", ctypes.c_int64), ("tile_bytes_cap", ctypes.c_int64),
                ("arena_grows", ctypes.c_int32), ("splitk_launches", ctypes.c_int32),
                ("qr_tiles_reg", ctypes.c_int32), ("qr_tiles_lds", ctypes.c_int32),
                ("qr_tiles_global", ctypes.c_int32), ("reserved_info", ctypes.c_int32),
                ("fp32_err_bound", ctypes.c_double)]


class KStat(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("ms", ctypes.c_double), ("flops", ctypes.c_double),
                ("bytes", ctypes.c_double)]


KCLASSES = ["update", "lowrank", "compress", "diag", "solve", "gradq", "gen"]

EXPORTS = ["tlr_create", "tlr_destroy", "tlr_generate", "tlr_compress", "tlr_potrf", "tlr_loglik",
           "tlr_loglik_grad", "tlr_get_ranks", "tlr_get_tangent_ranks", "tlr_get_info", "tlr_get_tile",
           "tlr_covariance_block", "tlr_morton_order", "tlr_last_error", "tlr_sample", "tlr_profile",
           "tlr_get_kstats", "tlr_loglik_grad_batched", "tlr_predict", "tlr_dense_loglik_noalloc",
           "tlr_loglik_grad3"]

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load the HIP library; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1804_09137_amd.build`")
    # torch must bring in its HIP runtime first: the library then binds to the
    # same libamdhip64 (same soname) instead of loading a second runtime.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    I64 = ctypes.c_int64
    D3 = ctypes.POINTER(ctypes.c_double)
    sig = {
        "tlr_create": [ctypes.POINTER(P), ctypes.POINTER(Opts), P],
        "tlr_destroy": [P],
        "tlr_generate": [P, P, P, D3],
        "tlr_compress": [P],
        "tlr_potrf": [P, ctypes.POINTER(I64)],
        "tlr_loglik": [P, P, D3, D3, D3],
        "tlr_loglik_grad": [P, P, P, P, D3, D3, D3, ctypes.POINTER(I64)],
        "tlr_loglik_grad3": [P, P, P, P, D3, D3, D3, ctypes.POINTER(I64)],
        "tlr_get_ranks": [P, ctypes.POINTER(ctypes.c_int32)],
        "tlr_get_tangent_ranks": [P, ctypes.POINTER(ctypes.c_int32)],
        "tlr_predict": [P, P, ctypes.c_int64, P, P, P, P],
        "tlr_dense_loglik_noalloc": [I64, P, P, P, D3, D3, D3, D3, ctypes.POINTER(I64), P],
        "tlr_get_info": [P, ctypes.POINTER(Info)],
        "tlr_get_tile": [P, ctypes.c_int32, ctypes.c_int32, P, I64],
        "tlr_covariance_block": [P, I64, I64, I64, I64, ctypes.c_int32, P, I64],
        "tlr_morton_order": [I64, D3, D3, ctypes.POINTER(I64)],
        "tlr_sample": [P, P, P],
        "tlr_profile": [P, ctypes.c_int32],
        "tlr_get_kstats": [P, ctypes.POINTER(KStat)],
        "tlr_loglik_grad_batched": [ctypes.c_int32, ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(P),
                                    ctypes.POINTER(P), D3, D3, D3, ctypes.POINTER(I64),
                                    ctypes.POINTER(ctypes.c_int32), ctypes.c_int32],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.tlr_last_error.argtypes = []
    lib.tlr_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def status_name(st: int) -> str:
    return _NAMES.get(st, f"status {st}")
