"""ctypes wrappers of the oracle's plain-C FP64 O(n) pass (test infrastructure).

Every input is converted to contiguous float64 first (float32 inputs convert
exactly), so the C code always computes in FP64.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def lib_path() -> str:
    return os.path.join(_HERE, "liboracle.so")


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(lib_path()):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(lib_path())
        p = ctypes.c_void_p
        i64 = ctypes.c_int64
        L.oracle_stencils.argtypes = [ctypes.c_int, p, p, p, p, i64, p, p, p, p]
        L.oracle_precompute.argtypes = [ctypes.c_int, p, p, p, p, p, i64, p, p, p, p]
        L.oracle_precompute_abs.argtypes = [ctypes.c_int, p, p, p, p, p, i64, p, p, p, p]
        L.oracle_probe_sketches.argtypes = [ctypes.c_int, p, p, p, p, i64,
                                            ctypes.c_uint64, ctypes.c_int, p, p]
        L.oracle_probe_value.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]
        L.oracle_probe_value.restype = ctypes.c_double
        L.oracle_splitmix64.argtypes = [ctypes.c_uint64]
        L.oracle_splitmix64.restype = ctypes.c_uint64
        L.oracle_interpolate.argtypes = [ctypes.c_int, p, p, p, p, p, i64, p, p]
        L.oracle_wtw_matvec.argtypes = [ctypes.c_int, p, p, p, p, ctypes.c_int]
        L.oracle_precompute_omp.argtypes = [ctypes.c_int, p, p, p, p, p, i64, p, p, p, p,
                                            ctypes.c_int]
        L.oracle_precompute_omp.restype = ctypes.c_int
        L.oracle_wtw_matvec_omp.argtypes = [ctypes.c_int, p, p, p, p, ctypes.c_int, ctypes.c_int]
        L.oracle_wtw_matvec_omp.restype = None
        L.oracle_set_interp.argtypes = [ctypes.c_int]
        L.oracle_set_interp.restype = None
        for f in (L.oracle_stencils, L.oracle_precompute, L.oracle_precompute_abs,
                  L.oracle_probe_sketches,
                  L.oracle_interpolate):
            f.restype = ctypes.c_int
        _LIB = L
    return _LIB


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


INTERP = {"cubic": 0, "linear": 1}


def _grid_arrays(grid):
    """Grid geometry as C arrays; also selects the interpolation scheme
    (grid["interp"]: "cubic" (default) or "linear") for the next C call."""
    _lib().oracle_set_interp(INTERP[grid.get("interp", "cubic")])
    d = grid["d"]
    m = np.ascontiguousarray(np.array(grid["m"][:d], dtype=np.int64))
    g0 = np.ascontiguousarray(np.array(grid["origin"][:d], dtype=np.float64))
    h = np.ascontiguousarray(np.array(grid["spacing"][:d], dtype=np.float64))
    return d, m, g0, h


def _coords(x, d):
    """x: a [d, n] array, a sequence of d length-n arrays, or (d = 1) one
    length-n array -> contiguous float64 [d][n]."""
    if isinstance(x, np.ndarray) and x.ndim == 1:
        X = x.astype(np.float64).reshape(1, -1)
    elif isinstance(x, np.ndarray):
        X = x.astype(np.float64).reshape(d, -1)
    else:
        X = np.stack([np.asarray(c, dtype=np.float64).reshape(-1) for c in x])
    assert X.shape[0] == d
    return np.ascontiguousarray(X)


class OutOfGrid(ValueError):
    pass


def _check(rc, bad):
    if rc == -2:
        raise OutOfGrid(f"point {int(bad.value)} lies outside the interpolable region")
    if rc != 0:
        raise ValueError(f"oracle call failed with status {rc}")


def stencils(grid, x):
    """Per-point stencil: (nodes [n,4^d] int64, weights [n,4^d], cell [n])."""
    d, m, g0, h = _grid_arrays(grid)
    X = _coords(x, d)
    n = X.shape[1]
    s = 4 ** d
    nodes = np.zeros((n, s), np.int64)
    w = np.zeros((n, s), np.float64)
    cells = np.zeros(n, np.int64)
    bad = ctypes.c_int64(-1)
    rc = _lib().oracle_stencils(d, _ptr(m), _ptr(g0), _ptr(h), _ptr(X), n,
                                _ptr(nodes), _ptr(w), _ptr(cells), ctypes.byref(bad))
    _check(rc, bad)
    return nodes, w, cells


def precompute(grid, x, y, absolute=False, threads=1):
    """Sufficient statistics (W^T W in [M, 7^d] stencil-diagonal layout,
    W^T y [M], y^T y), accumulated serially in FP64 in input order.  With
    `absolute`, the same sums over |w| and |y| (|W|^T |W|, |W|^T |y|): the
    scale of the rounding error of any summation order, for error bounds.
    threads > 1: the OpenMP variant (contiguous point chunks per thread,
    combined in thread order; deterministic per thread count)."""
    d, m, g0, h = _grid_arrays(grid)
    X = _coords(x, d)
    n = X.shape[1]
    Y = np.ascontiguousarray(np.asarray(y, dtype=np.float64).reshape(-1))
    assert Y.shape[0] == n
    M = int(np.prod(m))
    wtw = np.zeros((M, 7 ** d), np.float64)
    wty = np.zeros(M, np.float64)
    yty = ctypes.c_double(0.0)
    bad = ctypes.c_int64(-1)
    if threads > 1 and not absolute:
        rc = _lib().oracle_precompute_omp(d, _ptr(m), _ptr(g0), _ptr(h), _ptr(X), _ptr(Y), n,
                                          _ptr(wtw), _ptr(wty), ctypes.byref(yty),
                                          ctypes.byref(bad), int(threads))
    else:
        fn = _lib().oracle_precompute_abs if absolute else _lib().oracle_precompute
        rc = fn(d, _ptr(m), _ptr(g0), _ptr(h), _ptr(X), _ptr(Y), n,
                _ptr(wtw), _ptr(wty), ctypes.byref(yty), ctypes.byref(bad))
    _check(rc, bad)
    return wtw, wty, float(yty.value)


def splitmix64(z):
    return int(_lib().oracle_splitmix64(ctypes.c_uint64(z)))


def probe_values(seed, j, n):
    """Rademacher probe z_j[0..n) from the SplitMix64 counter generator."""
    L = _lib()
    return np.array([L.oracle_probe_value(seed, j, i) for i in range(n)], np.float64)


def probe_sketches(grid, x, seed, nprobe):
    """W^T z_j for j < nprobe: [nprobe, M]."""
    d, m, g0, h = _grid_arrays(grid)
    X = _coords(x, d)
    n = X.shape[1]
    M = int(np.prod(m))
    out = np.zeros((nprobe, M), np.float64)
    bad = ctypes.c_int64(-1)
    rc = _lib().oracle_probe_sketches(d, _ptr(m), _ptr(g0), _ptr(h), _ptr(X), n,
                                      ctypes.c_uint64(seed), nprobe, _ptr(out),
                                      ctypes.byref(bad))
    _check(rc, bad)
    return out


def interpolate(grid, mu_grid, xq):
    d, m, g0, h = _grid_arrays(grid)
    X = _coords(xq, d)
    nq = X.shape[1]
    mu = np.ascontiguousarray(np.asarray(mu_grid, np.float64).reshape(-1))
    out = np.zeros(nq, np.float64)
    bad = ctypes.c_int64(-1)
    rc = _lib().oracle_interpolate(d, _ptr(m), _ptr(g0), _ptr(h), _ptr(mu), _ptr(X), nq,
                                   _ptr(out), ctypes.byref(bad))
    _check(rc, bad)
    return out


def wtw_matvec(grid, wtw, v, threads=1):
    """u = (W^T W) v; v is [M] or [k, M] (threads > 1: rows split between
    OpenMP threads, same result)."""
    d, m, g0, h = _grid_arrays(grid)
    V = np.ascontiguousarray(np.asarray(v, np.float64))
    squeeze = V.ndim == 1
    V = V.reshape(-1, int(np.prod(m)))
    U = np.zeros_like(V)
    A = np.ascontiguousarray(wtw, np.float64)
    if threads > 1:
        _lib().oracle_wtw_matvec_omp(d, _ptr(m), _ptr(A), _ptr(V), _ptr(U), V.shape[0],
                                     int(threads))
    else:
        _lib().oracle_wtw_matvec(d, _ptr(m), _ptr(A), _ptr(V), _ptr(U), V.shape[0])
    return U[0] if squeeze else U
