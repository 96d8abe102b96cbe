"""CPU-only checks of the C ABI: every function include/fkgp.h declares is
exported by the built library, host-side argument validation rejects bad
input before touching a device, and the binding fails loudly without the
library (no CPU fallback)."""
import ctypes
import os
import re

import pytest

import paper_2101_11751_amd as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "fkgp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fkgp_[A-Za-z_]+)\s*\(", src)))


def test_header_declares_binding_exports():
    assert set(declared_functions()) == set(P.EXPORTS)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(P.LIB_PATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(P.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_host_validation_without_device():
    if not os.path.exists(P.LIB_PATH):
        pytest.skip("library not built")
    L = P.load_library()
    out = ctypes.c_void_p()
    g = P._Grid()
    g.d = 0
    assert L.fkgp_precompute(ctypes.byref(g), None, None, 0, 0, None, None,
                             ctypes.byref(out)) == P.EINVAL
    assert b"grid.d" in L.fkgp_last_error()
    g.d = 2
    g.m[0], g.m[1] = 3, 10
    g.spacing[0] = g.spacing[1] = 0.1
    assert L.fkgp_precompute(ctypes.byref(g), None, None, 0, 0, None, None,
                             ctypes.byref(out)) == P.EINVAL
    g.m[0] = 10
    assert L.fkgp_precompute(ctypes.byref(g), None, None, -5, 0, None, None,
                             ctypes.byref(out)) == P.EINVAL
    g.spacing[1] = -1.0
    assert L.fkgp_precompute(ctypes.byref(g), None, None, 0, 0, None, None,
                             ctypes.byref(out)) == P.EINVAL
    g.spacing[1] = 0.1
    # n > 0 requires pointers
    assert L.fkgp_precompute(ctypes.byref(g), None, None, 10, 0, None, None,
                             ctypes.byref(out)) == P.EINVAL
    # grid lines longer than the line FFT supports (circulant > 131072 points)
    g.m[1] = 65537
    assert L.fkgp_precompute(ctypes.byref(g), None, None, 0, 0, None, None,
                             ctypes.byref(out)) == P.EINVAL
    assert b"65536" in L.fkgp_last_error()
    assert L.fkgp_precompute(ctypes.byref(g), None, None, 0, 0, None, None, None) == P.EINVAL
    d = P._Desc()
    assert L.fkgp_describe(None, ctypes.byref(d)) == P.EINVAL
    assert L.fkgp_solve(None, None, None, None, None, None, None) == P.EINVAL
    assert L.fkgp_mll_and_grad(None, None, None, None, None, None, None) == P.EINVAL


def test_binding_fails_loudly_without_library(monkeypatch):
    monkeypatch.setattr(P, "_lib", None)
    monkeypatch.setattr(P, "LIB_PATH", "/nonexistent/libfkgp.so")
    with pytest.raises(ImportError):
        P.load_library()


def test_load_rejects_bad_files(tmp_path):
    """fkgp_load checks the file before touching the device: a missing file,
    another kind of file and a truncated header give FKGP_EINVAL."""
    L = P.load_library()
    out = ctypes.c_void_p()
    assert L.fkgp_load(str(tmp_path / "missing.bin").encode(), None, ctypes.byref(out)) == P.EINVAL
    assert out.value is None
    junk = tmp_path / "junk.bin"
    junk.write_bytes(b"not a statistics file" * 10)
    assert L.fkgp_load(str(junk).encode(), None, ctypes.byref(out)) == P.EINVAL
    assert b"statistics file" in L.fkgp_last_error()
    short = tmp_path / "short.bin"
    short.write_bytes(b"FKGPSTAT")
    assert L.fkgp_load(str(short).encode(), None, ctypes.byref(out)) == P.EINVAL
    assert L.fkgp_save(None, b"x", None) == P.EINVAL
    assert P._STATS_HEADER.size == 136


def test_allocator_validation_without_device():
    """fkgp_set_allocator: NULL restores the default; a table without both
    functions is rejected."""
    if not os.path.exists(P.LIB_PATH):
        pytest.skip("library not built")
    L = P.load_library()
    assert L.fkgp_set_allocator(None) == P.OK
    bad = P._Allocator()
    assert L.fkgp_set_allocator(ctypes.byref(bad)) == P.EINVAL
    assert b"alloc and free" in L.fkgp_last_error()
    assert L.fkgp_set_allocator(None) == P.OK


def test_new_entry_points_validate_on_the_host():
    """The covariance, rank-k, multi-right-hand-side and exact-trace entry
    points reject NULL handles and bad sizes before touching a device."""
    if not os.path.exists(P.LIB_PATH):
        pytest.skip("library not built")
    L = P.load_library()
    hyp = P._Hypers()
    info = P._SolveInfo()
    cov = ctypes.c_void_p(1)
    assert L.fkgp_posterior_cov(None, ctypes.byref(hyp), None, 4, P.F64, 1e-8, 10, cov,
                                ctypes.byref(info), None) == P.EINVAL
    out = ctypes.c_void_p()
    assert L.fkgp_love_build(None, ctypes.byref(hyp), 10, None, ctypes.byref(out)) == P.EINVAL
    assert out.value is None
    assert L.fkgp_love_build(None, ctypes.byref(hyp), 10, None, None) == P.EINVAL
    r = ctypes.c_int(0)
    assert L.fkgp_love_tridiag(None, ctypes.byref(r), None, None, None) == P.EINVAL
    assert L.fkgp_love_cov(None, None, 1, P.F64, None, None) == P.EINVAL
    L.fkgp_love_destroy(None)
    assert L.fkgp_solve_multi(None, ctypes.byref(hyp), None, 3, None, None, None,
                              None) == P.EINVAL
    opts = P._MllOpts(30, 1e-6, 1000, 1, 0, 0, 1)
    mll = ctypes.c_double()
    grad = (ctypes.c_double * 5)()
    assert L.fkgp_mll_and_grad(None, ctypes.byref(hyp), ctypes.byref(opts), ctypes.byref(mll),
                               grad, None, None) == P.EINVAL


def test_streamed_precompute_validates_on_the_host():
    """fkgp_precompute_host rejects kept points and out-of-range probe
    counts before touching a device (probe sketches themselves are allowed)."""
    if not os.path.exists(P.LIB_PATH):
        pytest.skip("library not built")
    L = P.load_library()
    g = P._Grid()
    g.d = 1
    g.m[0] = 50
    g.spacing[0] = 0.02
    out = ctypes.c_void_p()
    keep = P._PreOpts(P.F32, 0, 0, 1, 0)
    assert L.fkgp_precompute_host(ctypes.byref(g), None, None, 0, P.F32, ctypes.byref(keep), 0,
                                  None, ctypes.byref(out)) == P.EINVAL
    assert b"keeps no points" in L.fkgp_last_error()
    many = P._PreOpts(P.F32, 32, 0, 0, 0)
    assert L.fkgp_precompute_host(ctypes.byref(g), None, None, 0, P.F32, ctypes.byref(many), 0,
                                  None, ctypes.byref(out)) == P.EINVAL
    assert b"n_probes" in L.fkgp_last_error()
    assert out.value is None
