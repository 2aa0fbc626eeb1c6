"""CPU checks of the C-ABI library: it loads, exports every symbol the header
declares, validates arguments before touching the GPU, and its host Morton
helper reproduces the oracle's ordering bit for bit."""
import ctypes
import os
import re

import numpy as np
import pytest

import synth
from oracle import ordering as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_1804_09137_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libtlrmle.so not built (run __graft_entry__.build())")
    return _lib, _lib.load()


def test_missing_library_raises(monkeypatch, tmp_path):
    # no CPU fallback: without the built library the binding refuses to load
    from paper_1804_09137_amd import _lib as m
    monkeypatch.setattr(m, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        m.load(str(tmp_path / "libtlrmle.so"))


def test_short_tensors_are_refused_before_any_call():
    # the C-ABI takes bare pointers: the binding checks lengths on the host
    import torch
    from paper_1804_09137_amd import _check_len
    _check_len(torch.zeros(5, dtype=torch.float64), 5)
    _check_len(torch.zeros(6, dtype=torch.float64), 5)
    with pytest.raises(ValueError, match="z: expected at least 5 elements, got 4"):
        _check_len(torch.zeros(4, dtype=torch.float64), 5, "z")


def test_header_symbols_exported():
    _m, lib = _lib()
    header = open(os.path.join(ROOT, "include", "tlr.h")).read()
    declared = set(re.findall(r"^(?:tlr_status|const char\*)\s+(tlr_\w+)\s*\(", header, flags=re.M))
    assert declared == set(_m.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name


def test_create_rejects_bad_options_without_gpu():
    m, lib = _lib()
    h = ctypes.c_void_p()
    bad = [dict(n=0, nb=64, tol=1e-9), dict(n=100, nb=40, tol=1e-9), dict(n=100, nb=2048, tol=1e-9),
           dict(n=100, nb=64, tol=0.0), dict(n=100, nb=64, tol=float("nan")),
           dict(n=100, nb=64, tol=1e-9, mode=7), dict(n=100, nb=64, tol=1e-9, mode=1, prec=1)]
    for kw in bad:
        o = m.Opts()
        o.n, o.nb, o.tol = kw["n"], kw["nb"], kw["tol"]
        o.mode, o.prec = kw.get("mode", 0), kw.get("prec", 0)
        assert lib.tlr_create(ctypes.byref(h), ctypes.byref(o), None) == m.TLR_EINVAL
    assert lib.tlr_create(None, None, None) == m.TLR_EINVAL
    assert lib.tlr_destroy(None) == m.TLR_OK
    assert lib.tlr_potrf(None, None) == m.TLR_EINVAL
    assert lib.tlr_loglik(None, None, None, None, None) == m.TLR_EINVAL
    assert lib.tlr_predict(None, None, 0, None, None, None, None) == m.TLR_EINVAL
    for kw in (dict(metric=2), dict(arena_bytes=-1), dict(sphere_radius=float("nan"))):
        o = m.Opts()
        o.n, o.nb, o.tol = 100, 64, 1e-9
        for k, v in kw.items():
            setattr(o, k, v)
        assert lib.tlr_create(ctypes.byref(h), ctypes.byref(o), None) == m.TLR_EINVAL


def test_noalloc_rejects_sizes_without_gpu():
    # argument checks come before any GPU call
    m, lib = _lib()
    D3 = ctypes.c_double * 3
    fake = ctypes.c_void_p(16)
    th = D3(1.0, 0.1, 0.5)
    assert lib.tlr_dense_loglik_noalloc(100, None, fake, fake, th, None, None, None, None, None) == m.TLR_EINVAL
    assert lib.tlr_dense_loglik_noalloc(0, fake, fake, fake, th, None, None, None, None, None) == m.TLR_EINVAL
    assert lib.tlr_dense_loglik_noalloc(2049, fake, fake, fake, th, None, None, None, None, None) == m.TLR_EINVAL
    assert b"exceeds the maximum 2048" in lib.tlr_last_error()


@pytest.mark.parametrize("m,seed", [(40, 0), (57, 3), (200, 0)])
def test_morton_matches_oracle(m, seed):
    from paper_1804_09137_amd import morton_order
    _lib()
    x, y = synth.jittered_grid(m, seed)
    np.testing.assert_array_equal(morton_order(x, y), O.morton_order(x, y))


def test_morton_edge_cases():
    from paper_1804_09137_amd import morton_order
    _lib()
    assert morton_order(np.array([0.3]), np.array([0.7])).tolist() == [0]
    x = np.array([0.5, 0.5, 0.5, 0.5])
    y = np.array([0.2, 0.1, 0.2, 0.1])
    np.testing.assert_array_equal(morton_order(x, y), O.morton_order(x, y))
    x, y = synth.jittered_subset(2345, seed=4)
    np.testing.assert_array_equal(morton_order(x, y), O.morton_order(x, y))


def test_struct_layouts_match_the_header(tmp_path):
    """The ctypes mirrors of tlr_opts, tlr_info and tlr_kstat have the sizes
    and field offsets a C compiler gives the header's structs."""
    import shutil
    import subprocess
    from paper_1804_09137_amd import _lib as m
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"tlr_opts": m.Opts, "tlr_info": m.Info, "tlr_kstat": m.KStat}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "tlr.h"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict((" ".join(l.split()[:2]), int(l.split()[2]))
               for l in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines())
    for cname, cls in structs.items():
        assert got[f"{cname} size"] == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[f"{cname} {fname}"] == getattr(cls, fname).offset, (cname, fname)
