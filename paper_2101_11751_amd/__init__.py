"""Python binding of libfkgp, the MI355X (gfx950) implementation of the hot path
of "Faster Kernel Interpolation for Gaussian Processes" (Yadav, Sheldon,
Musco): the one-shot O(n) sufficient-statistics pass and the n-independent
factorized conjugate-gradient operator (banded W^T W product composed with the
Kronecker-of-Toeplitz grid kernel through circulant-embedding FFTs).

This module only marshals arguments: torch provides device memory and the
current stream, and every step runs in the HIP kernels of ``libfkgp.so`` (the
C ABI of ``include/fkgp.h``).  There is no CPU fallback: if the library has
not been built, every entry point raises.
"""
import ctypes
import math
import os
import struct

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfkgp.so")

F32, F64 = 0, 1
OK, ENOTCONV, EINVAL, EOUTOFGRID, ENOMEM, EDEVICE = 0, 1, -1, -2, -3, -4

#: every symbol that include/fkgp.h declares
EXPORTS = ("fkgp_precompute", "fkgp_describe", "fkgp_export_stats", "fkgp_export_sketches",
           "fkgp_solve", "fkgp_solve_noalloc", "fkgp_solve_multi", "fkgp_mll_and_grad", "fkgp_batch_mll_and_grad", "fkgp_interpolate",
           "fkgp_posterior_cov", "fkgp_love_build", "fkgp_love_tridiag", "fkgp_love_cov",
           "fkgp_love_destroy", "fkgp_apply_B",
           "fkgp_kg_matvec", "fkgp_wtw_matvec", "fkgp_wtw_matvec_dot", "fkgp_ski_solve", "fkgp_save", "fkgp_load",
           "fkgp_precompute_host", "fkgp_set_allocator", "fkgp_destroy", "fkgp_last_error")


class FkgpError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"fkgp status {status}: {msg}")
        self.status = status


class OutOfGridError(FkgpError, ValueError):
    pass


class _Grid(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int), ("m", ctypes.c_int64 * 3),
                ("origin", ctypes.c_double * 3), ("spacing", ctypes.c_double * 3)]


class _Hypers(ctypes.Structure):
    _fields_ = [("lengthscale", ctypes.c_double * 3), ("outputscale", ctypes.c_double),
                ("noise_std", ctypes.c_double), ("kernel", ctypes.c_int)]


# fkgp_kernel: the one-dimensional kernel of the product (hypers["kernel"])
KERNELS = {"se": 0, "matern12": 1, "matern32": 2, "matern52": 3}


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class _Allocator(ctypes.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("ctx", ctypes.c_void_p)]


class _PreOpts(ctypes.Structure):
    _fields_ = [("stats_dtype", ctypes.c_int), ("n_probes", ctypes.c_int),
                ("probe_seed", ctypes.c_uint64), ("keep_points", ctypes.c_int),
                ("interp", ctypes.c_int)]


#: interpolation schemes (fkgp_interp); a grid dict selects one with "interp"
INTERP = {"cubic": 0, "linear": 1}


def _interp_code(grid):
    return INTERP[grid.get("interp", "cubic")]


class _Desc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m_total", ctypes.c_int64), ("d", ctypes.c_int),
                ("stats_dtype", ctypes.c_int), ("n_probes", ctypes.c_int),
                ("yty", ctypes.c_double), ("bytes_wtw", ctypes.c_int64),
                ("nnz_wtw", ctypes.c_int64), ("halo", ctypes.c_int64),
                ("wtw_blocks", ctypes.c_int64), ("wtw_blocks_nonzero", ctypes.c_int64),
                ("wtw_block_entries", ctypes.c_int64), ("interp", ctypes.c_int),
                ("nnz_wtw_nonzero", ctypes.c_int64)]


OP_F64, OP_STATS = 0, 1


class _SolveOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("maxiter", ctypes.c_int),
                ("op_precision", ctypes.c_int)]


class _SolveInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("converged", ctypes.c_int),
                ("rel_residual", ctypes.c_double)]


class _MllOpts(ctypes.Structure):
    _fields_ = [("lanczos_steps", ctypes.c_int), ("tol", ctypes.c_double),
                ("maxiter", ctypes.c_int), ("batched", ctypes.c_int),
                ("batch_rhs", ctypes.c_int), ("batch_block", ctypes.c_int),
                ("trace_mode", ctypes.c_int)]


class _MllInfo(ctypes.Structure):
    _fields_ = [("logdet", ctypes.c_double), ("quad", ctypes.c_double),
                ("iterations_y", ctypes.c_int), ("iterations_probes_max", ctypes.c_int),
                ("batch_rhs", ctypes.c_int), ("batch_block", ctypes.c_int),
                ("dquad", ctypes.c_double * 5)]


_lib = None


def load_library():
    """Loads libfkgp.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2101_11751_amd.build` (no CPU fallback exists)")
    L = ctypes.CDLL(LIB_PATH)
    p = ctypes.c_void_p
    L.fkgp_precompute.argtypes = [ctypes.POINTER(_Grid), ctypes.POINTER(p), p, ctypes.c_int64,
                                  ctypes.c_int, ctypes.POINTER(_PreOpts), p, ctypes.POINTER(p)]
    L.fkgp_describe.argtypes = [p, ctypes.POINTER(_Desc)]
    L.fkgp_export_stats.argtypes = [p, p, p, ctypes.POINTER(ctypes.c_double), p]
    L.fkgp_export_sketches.argtypes = [p, p, p]
    L.fkgp_solve.argtypes = [p, ctypes.POINTER(_Hypers), p, p, ctypes.POINTER(_SolveOpts),
                             ctypes.POINTER(_SolveInfo), p]
    L.fkgp_solve_noalloc.argtypes = [p, ctypes.POINTER(_Hypers), p, p,
                                     ctypes.POINTER(_SolveOpts), ctypes.POINTER(_SolveInfo), p]
    L.fkgp_precompute_host.argtypes = [ctypes.POINTER(_Grid), ctypes.POINTER(p), p,
                                       ctypes.c_int64, ctypes.c_int, ctypes.POINTER(_PreOpts),
                                       ctypes.c_int64, p, ctypes.POINTER(p)]
    L.fkgp_save.argtypes = [p, ctypes.c_char_p, p]
    L.fkgp_load.argtypes = [ctypes.c_char_p, p, ctypes.POINTER(ctypes.c_void_p)]
    L.fkgp_solve_multi.argtypes = [p, ctypes.POINTER(_Hypers), p, ctypes.c_int, p,
                                   ctypes.POINTER(_SolveOpts), ctypes.POINTER(_SolveInfo), p]
    L.fkgp_ski_solve.argtypes = [p, ctypes.POINTER(_Hypers), ctypes.c_double, ctypes.c_int, p,
                                 ctypes.POINTER(_SolveInfo), p]
    L.fkgp_mll_and_grad.argtypes = [p, ctypes.POINTER(_Hypers), ctypes.POINTER(_MllOpts),
                                    ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_MllInfo), p]
    L.fkgp_batch_mll_and_grad.argtypes = [ctypes.POINTER(p), ctypes.c_int,
                                          ctypes.POINTER(_Hypers), ctypes.POINTER(_MllOpts),
                                          ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(_MllInfo), p]
    L.fkgp_interpolate.argtypes = [p, p, ctypes.POINTER(p), ctypes.c_int64, ctypes.c_int, p, p]
    L.fkgp_love_build.argtypes = [p, ctypes.POINTER(_Hypers), ctypes.c_int, p,
                                  ctypes.POINTER(ctypes.c_void_p)]
    L.fkgp_love_tridiag.argtypes = [p, ctypes.POINTER(ctypes.c_int), p, p, p]
    L.fkgp_love_cov.argtypes = [p, ctypes.POINTER(p), ctypes.c_int64, ctypes.c_int, p, p]
    L.fkgp_love_destroy.argtypes = [p]
    L.fkgp_love_destroy.restype = None
    L.fkgp_posterior_cov.argtypes = [p, ctypes.POINTER(_Hypers), ctypes.POINTER(p), ctypes.c_int64,
                                     ctypes.c_int, ctypes.c_double, ctypes.c_int, p,
                                     ctypes.POINTER(_SolveInfo), p]
    L.fkgp_apply_B.argtypes = [p, ctypes.POINTER(_Hypers), p, p, p, ctypes.c_int, p]
    L.fkgp_kg_matvec.argtypes = [p, ctypes.POINTER(_Hypers), p, p, ctypes.c_int, p]
    L.fkgp_wtw_matvec.argtypes = [p, p, p, ctypes.c_int, ctypes.c_int, p]
    L.fkgp_wtw_matvec_dot.argtypes = [p, p, p, ctypes.c_int, p, ctypes.c_int, p]
    L.fkgp_set_allocator.argtypes = [ctypes.POINTER(_Allocator)]
    L.fkgp_destroy.argtypes = [p]
    L.fkgp_destroy.restype = None
    L.fkgp_last_error.argtypes = []
    L.fkgp_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("fkgp_destroy", "fkgp_last_error"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(status):
    if status == OK:
        return status
    msg = load_library().fkgp_last_error().decode()
    if status == ENOTCONV:
        return status
    if status == EOUTOFGRID:
        raise OutOfGridError(status, msg)
    raise FkgpError(status, msg)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _grid_struct(grid):
    g = _Grid()
    g.d = int(grid["d"])
    for k in range(g.d):
        g.m[k] = int(grid["m"][k])
        g.origin[k] = float(grid["origin"][k])
        g.spacing[k] = float(grid["spacing"][k])
    return g


def _hyp_struct(hyp, d):
    h = _Hypers()
    ell = hyp["lengthscale"]
    ell = list(ell) if hasattr(ell, "__len__") else [ell] * d
    for k in range(d):
        h.lengthscale[k] = float(ell[k])
    h.outputscale = float(hyp["outputscale"])
    h.noise_std = float(hyp["noise"])
    kind = hyp.get("kernel", "se")
    h.kernel = KERNELS[kind] if isinstance(kind, str) else int(kind)
    return h


def _dtype_code(t):
    if t == torch.float32:
        return F32
    if t == torch.float64:
        return F64
    raise TypeError(f"unsupported dtype {t}")


class Handle:
    """Sufficient statistics of one data set on one device (immutable)."""

    def __init__(self, ptr, grid):
        self._ptr = ptr
        self.grid = grid
        d = _Desc()
        _check(load_library().fkgp_describe(ptr, ctypes.byref(d)))
        self.n = d.n
        self.m_total = d.m_total
        self.d = d.d
        self.stats_dtype = torch.float32 if d.stats_dtype == F32 else torch.float64
        self.n_probes = d.n_probes
        self.yty = d.yty
        self.bytes_wtw = d.bytes_wtw
        self.nnz_wtw = d.nnz_wtw
        self.halo = d.halo
        self.wtw_blocks = d.wtw_blocks
        self.wtw_blocks_nonzero = d.wtw_blocks_nonzero
        self.wtw_block_entries = d.wtw_block_entries
        self.nnz_wtw_nonzero = d.nnz_wtw_nonzero
        self.interp = "linear" if d.interp == INTERP["linear"] else "cubic"

    @property
    def ptr(self):
        return self._ptr

    def close(self):
        if self._ptr:
            load_library().fkgp_destroy(self._ptr)
            self._ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def precompute(grid, x, y, stats_dtype=torch.float32, n_probes=0, probe_seed=0,
               keep_points=False):
    """fkgp_precompute: x is a list of d device tensors (float32 or float64),
    y a device tensor of the same dtype and length.  keep_points: also keep
    the points in cell order for ski_solve (d <= 2)."""
    L = load_library()
    d = int(grid["d"])
    xs = [t.contiguous() for t in x]
    y = y.contiguous()
    n = y.numel()
    dt = _dtype_code(y.dtype)
    for t in xs:
        assert t.dtype == y.dtype and t.numel() == n and t.is_cuda
    arr = (ctypes.c_void_p * 3)(*([t.data_ptr() for t in xs] + [0] * (3 - d)))
    g = _grid_struct(grid)
    o = _PreOpts(_dtype_code(stats_dtype), int(n_probes), int(probe_seed), int(bool(keep_points)),
                 _interp_code(grid))
    out = ctypes.c_void_p()
    _check(L.fkgp_precompute(ctypes.byref(g), arr, _ptr(y), n, dt, ctypes.byref(o), _stream(),
                             ctypes.byref(out)))
    return Handle(out, grid)


def precompute_host(grid, x, y, stats_dtype=torch.float32, chunk=0, n_probes=0, probe_seed=0):
    """fkgp_precompute_host: x is a list of d host arrays (numpy or CPU
    tensors, float32 or float64), y a host array of the same dtype; the
    points stream to the device in chunks of `chunk` points (0: 2^24).
    n_probes / probe_seed: probe sketches as in `precompute`."""
    L = load_library()
    d = int(grid["d"])
    xs = [np.ascontiguousarray(t.numpy() if isinstance(t, torch.Tensor) else t) for t in x]
    yv = np.ascontiguousarray(y.numpy() if isinstance(y, torch.Tensor) else y)
    n = yv.shape[0]
    for t in xs:
        assert t.dtype == yv.dtype and t.shape == (n,)
    dt = F32 if yv.dtype == np.float32 else F64
    arr = (ctypes.c_void_p * 3)(*([t.ctypes.data for t in xs] + [0] * (3 - d)))
    g = _grid_struct(grid)
    o = _PreOpts(_dtype_code(stats_dtype), int(n_probes), int(probe_seed), 0, _interp_code(grid))
    out = ctypes.c_void_p()
    _check(L.fkgp_precompute_host(ctypes.byref(g), arr, yv.ctypes.data, n, dt, ctypes.byref(o),
                                  int(chunk), _stream(), ctypes.byref(out)))
    return Handle(out, grid)


def export_stats(h):
    """(W^T W [M, 7^d] canonical layout, W^T y [M] float64, y^T y)."""
    L = load_library()
    dev = torch.device("cuda", torch.cuda.current_device())
    wtw = torch.empty(h.m_total, 7 ** h.d, dtype=h.stats_dtype, device=dev)
    wty = torch.empty(h.m_total, dtype=torch.float64, device=dev)
    yty = ctypes.c_double()
    _check(L.fkgp_export_stats(h.ptr, _ptr(wtw), _ptr(wty), ctypes.byref(yty), _stream()))
    return wtw, wty, yty.value


def export_sketches(h):
    L = load_library()
    dev = torch.device("cuda", torch.cuda.current_device())
    out = torch.empty(h.n_probes, h.m_total, dtype=torch.float64, device=dev)
    _check(L.fkgp_export_sketches(h.ptr, _ptr(out), _stream()))
    return out


def solve(h, hypers, rhs=None, tol=1e-6, maxiter=1000, op_precision="f64", out=None,
          noalloc=False):
    """Posterior-mean grid weights mu_G (rhs None), or W^T A^{-1} W rhs.
    op_precision "f64": operator arithmetic in FP64 on the stored W^T W;
    "stats": arithmetic in the stats dtype (FP32 handles: FP32 inner CG with
    FP64 iterative refinement).  out: optional [M] float64 device tensor to
    write.  noalloc: fkgp_solve_noalloc (the library's fixed workspace, no
    allocation).  Returns (out [M] float64, info dict)."""
    L = load_library()
    dev = torch.device("cuda", torch.cuda.current_device())
    if out is None:
        out = torch.empty(h.m_total, dtype=torch.float64, device=dev)
    assert out.dtype == torch.float64 and out.is_contiguous() and out.numel() == h.m_total
    if rhs is not None:
        rhs = rhs.to(torch.float64).contiguous()
    info = _SolveInfo()
    fn = L.fkgp_solve_noalloc if noalloc else L.fkgp_solve
    st = _check(fn(h.ptr, ctypes.byref(_hyp_struct(hypers, h.d)), _ptr(rhs), _ptr(out),
                             ctypes.byref(_SolveOpts(float(tol), int(maxiter),
                                                     OP_STATS if op_precision == "stats"
                                                     else OP_F64)),
                             ctypes.byref(info), _stream()))
    return out, {"iterations": info.iterations, "converged": bool(info.converged),
                 "rel_residual": info.rel_residual, "status": st}


_ALLOCATOR_KEEPALIVE = None


def set_allocator(alloc=None, free=None):
    """fkgp_set_allocator: alloc(nbytes, stream) -> device pointer (int, 0 on
    failure) and free(ptr, stream) for the library's device memory; no
    arguments restore the default pool."""
    global _ALLOCATOR_KEEPALIVE
    L = load_library()
    if alloc is None:
        _check(L.fkgp_set_allocator(None))
        _ALLOCATOR_KEEPALIVE = None
        return
    a = _ALLOC_FN(lambda n, s, c: alloc(int(n), s) or None)
    f = _FREE_FN(lambda ptr, s, c: free(ptr, s))
    st = _Allocator(a, f, None)
    _check(L.fkgp_set_allocator(ctypes.byref(st)))
    _ALLOCATOR_KEEPALIVE = (a, f, st)


def torch_allocator():
    """(alloc, free) taking the library's device memory from torch's caching
    allocator on the current stream."""
    def alloc(n, stream):
        return torch.cuda.caching_allocator_alloc(n)

    def free(ptr, stream):
        torch.cuda.caching_allocator_delete(ptr)

    return alloc, free


def solve_multi(h, hypers, rhs, tol=1e-6, maxiter=1000):
    """fkgp_solve_multi: W^T A^{-1} W rhs_j for k grid right-hand sides
    (rhs [k, M]); returns (out [k, M] float64, info dict)."""
    L = load_library()
    R = rhs.to(torch.float64).reshape(-1, h.m_total).contiguous()
    out = torch.empty_like(R)
    info = _SolveInfo()
    st = _check(L.fkgp_solve_multi(h.ptr, ctypes.byref(_hyp_struct(hypers, h.d)), _ptr(R),
                                   R.shape[0], _ptr(out),
                                   ctypes.byref(_SolveOpts(float(tol), int(maxiter), OP_F64)),
                                   ctypes.byref(info), _stream()))
    return out, {"iterations": info.iterations, "converged": bool(info.converged),
                 "rel_residual": info.rel_residual, "status": st}


# header of a statistics file (fkgp_save): magic, version, d, m[3], origin[3],
# spacing[3], n, stats dtype, probes, probe seed, y^T y, nonzero blocks,
# interpolation scheme, reserved
_STATS_HEADER = struct.Struct("<8sIi3q3d3dqiiQdqii")


def save(h, path):
    """fkgp_save: write the handle's statistics to `path`."""
    _check(load_library().fkgp_save(h.ptr, os.fsencode(path), _stream()))


def load(path):
    """fkgp_load: a handle from a file written by save()."""
    L = load_library()
    out = ctypes.c_void_p()
    _check(L.fkgp_load(os.fsencode(path), _stream(), ctypes.byref(out)))
    with open(path, "rb") as f:
        hd = _STATS_HEADER.unpack(f.read(_STATS_HEADER.size))
    d = hd[2]
    grid = {"d": d, "m": list(hd[3:6])[:d], "origin": list(hd[6:9])[:d],
            "spacing": list(hd[9:12])[:d]}
    if hd[18] == INTERP["linear"]:
        grid["interp"] = "linear"
    return Handle(out, grid)


def ski_solve(h, hypers, tol=1e-6, maxiter=1000):
    """fkgp_ski_solve: the plain SKI baseline (CG in n-space on
    W K_G W^T + s2 I); returns (mean grid weights [M] float64, info dict)."""
    L = load_library()
    dev = torch.device("cuda", torch.cuda.current_device())
    out = torch.empty(h.m_total, dtype=torch.float64, device=dev)
    info = _SolveInfo()
    st = _check(L.fkgp_ski_solve(h.ptr, ctypes.byref(_hyp_struct(hypers, h.d)), float(tol),
                                 int(maxiter), _ptr(out), ctypes.byref(info), _stream()))
    return out, {"iterations": info.iterations, "converged": bool(info.converged),
                 "rel_residual": info.rel_residual, "status": st}


def interpolate(h, mean_grid, xq):
    L = load_library()
    xs = [t.contiguous() for t in xq]
    nq = xs[0].numel()
    out = torch.empty(nq, dtype=torch.float64, device=xs[0].device)
    arr = (ctypes.c_void_p * 3)(*([t.data_ptr() for t in xs] + [0] * (3 - len(xs))))
    _check(L.fkgp_interpolate(h.ptr, _ptr(mean_grid.contiguous()), arr, nq,
                              _dtype_code(xs[0].dtype), _ptr(out), _stream()))
    return out


def posterior_cov(h, hypers, xq, tol=1e-8, maxiter=1000):
    """fkgp_posterior_cov: SKI posterior covariance [nq, nq] (float64) between
    the query points xq (d device tensors of nq coordinates); returns
    (cov, info dict)."""
    L = load_library()
    xs = [t.contiguous() for t in xq]
    nq = xs[0].numel()
    out = torch.empty(nq, nq, dtype=torch.float64, device=xs[0].device)
    arr = (ctypes.c_void_p * 3)(*([t.data_ptr() for t in xs] + [0] * (3 - len(xs))))
    info = _SolveInfo()
    st = _check(L.fkgp_posterior_cov(h.ptr, ctypes.byref(_hyp_struct(hypers, h.d)), arr, nq,
                                     _dtype_code(xs[0].dtype), float(tol), int(maxiter),
                                     _ptr(out), ctypes.byref(info), _stream()))
    return out, {"iterations": info.iterations, "converged": bool(info.converged),
                 "rel_residual": info.rel_residual, "status": st}


class LoveCache:
    """Rank-k covariance cache (fkgp_love_build); `rank` is the number of
    Lanczos steps taken."""

    def __init__(self, ptr, d):
        self.ptr = ptr
        self.d = d
        L = load_library()
        r = ctypes.c_int(0)
        _check(L.fkgp_love_tridiag(ptr, ctypes.byref(r), None, None, None))
        self.rank = r.value

    def tridiag(self):
        """(alpha [rank], beta [rank-1], d [rank]) as float64 numpy arrays."""
        L = load_library()
        k = self.rank
        a = np.zeros(k)
        b = np.zeros(max(k - 1, 0))
        dd = np.zeros(k)
        r = ctypes.c_int(0)
        _check(L.fkgp_love_tridiag(self.ptr, ctypes.byref(r), a.ctypes.data_as(ctypes.c_void_p),
                                   b.ctypes.data_as(ctypes.c_void_p) if k > 1 else None,
                                   dd.ctypes.data_as(ctypes.c_void_p)))
        return a, b, dd

    def cov(self, xq):
        L = load_library()
        xs = [t.contiguous() for t in xq]
        nq = xs[0].numel()
        out = torch.empty(nq, nq, dtype=torch.float64, device=xs[0].device)
        arr = (ctypes.c_void_p * 3)(*([t.data_ptr() for t in xs] + [0] * (3 - len(xs))))
        _check(L.fkgp_love_cov(self.ptr, arr, nq, _dtype_code(xs[0].dtype), _ptr(out),
                               _stream()))
        return out

    def close(self):
        if self.ptr:
            load_library().fkgp_love_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def love_build(h, hypers, k):
    """fkgp_love_build: factorized Lanczos (k steps from y) and the rank-k
    covariance cache."""
    L = load_library()
    out = ctypes.c_void_p()
    _check(L.fkgp_love_build(h.ptr, ctypes.byref(_hyp_struct(hypers, h.d)), int(k), _stream(),
                             ctypes.byref(out)))
    return LoveCache(out, h.d)


def apply_B(h, hypers, x):
    """x: [k, M] (or [M]) in the handle's stats dtype -> (v, u)."""
    L = load_library()
    squeeze = x.dim() == 1
    X = x.reshape(-1, h.m_total).to(h.stats_dtype).contiguous()
    v = torch.empty_like(X)
    u = torch.empty_like(X)
    _check(L.fkgp_apply_B(h.ptr, ctypes.byref(_hyp_struct(hypers, h.d)), _ptr(X), _ptr(v),
                          _ptr(u), X.shape[0], _stream()))
    return (v[0], u[0]) if squeeze else (v, u)


def kg_matvec(h, hypers, x):
    L = load_library()
    squeeze = x.dim() == 1
    X = x.reshape(-1, h.m_total).to(h.stats_dtype).contiguous()
    out = torch.empty_like(X)
    _check(L.fkgp_kg_matvec(h.ptr, ctypes.byref(_hyp_struct(hypers, h.d)), _ptr(X), _ptr(out),
                            X.shape[0], _stream()))
    return out[0] if squeeze else out


def padded(h, x, dtype=None):
    """[k, M] (or [M]) -> zero-padded [k, M + 2 halo] buffer (stats dtype by
    default, or float64 for FP64 vectors against FP32-stored entries)."""
    X = x.reshape(-1, h.m_total)
    dt = dtype or h.stats_dtype
    out = torch.zeros(X.shape[0], h.m_total + 2 * h.halo, dtype=dt, device=X.device)
    out[:, h.halo:h.halo + h.m_total] = X
    return out


def wtw_matvec_padded(h, xpad, u):
    """u[k, M] = W^T W xpad (xpad from `padded`); launches one kernel, no sync."""
    _check(load_library().fkgp_wtw_matvec(h.ptr, _ptr(xpad), _ptr(u), xpad.shape[0],
                                          _dtype_code(xpad.dtype), _stream()))
    return u


def wtw_matvec_dot(h, xpad, u, reps=1):
    """fkgp_wtw_matvec_dot: u = (W^T W) x with u^T x reduced in the same launch
    (the product as the CG loop runs it), repeated `reps` times; xpad: one
    padded FP64 vector [1, M + 2 halo]; u: [1, M] float64.  Returns u^T x
    (a 1-element float64 device tensor)."""
    L = load_library()
    assert xpad.dtype == torch.float64 and u.dtype == torch.float64
    dot = torch.empty(1, dtype=torch.float64, device=u.device)
    _check(L.fkgp_wtw_matvec_dot(h.ptr, _ptr(xpad), _ptr(u), F64, _ptr(dot), int(reps),
                                 _stream()))
    return dot


def wtw_matvec(h, x, dtype=None):
    squeeze = x.dim() == 1
    xp = padded(h, x, dtype)
    u = torch.empty(xp.shape[0], h.m_total, dtype=xp.dtype, device=x.device)
    wtw_matvec_padded(h, xp, u)
    return u[0] if squeeze else u


def mll_and_grad(h, hypers, lanczos_steps=30, tol=1e-6, maxiter=1000, batched=True,
                 trace="hutchinson"):
    """(mll, grad [d+2] w.r.t. (log l_k, log s, log sigma), info).  batched:
    all probes advance together (one W^T W read per iteration).  trace:
    "hutchinson" (over the probes), "exact" (m grid solves, m <= 4096) or
    "slq" (the derivative of the returned Lanczos estimate itself)."""
    L = load_library()
    mll = ctypes.c_double()
    grad = (ctypes.c_double * (h.d + 2))()
    info = _MllInfo()
    tm = {"hutchinson": 0, "exact": 1, "slq": 2}[trace]
    st = _check(L.fkgp_mll_and_grad(h.ptr, ctypes.byref(_hyp_struct(hypers, h.d)),
                                    ctypes.byref(_MllOpts(int(lanczos_steps), float(tol),
                                                          int(maxiter), int(bool(batched)), 0, 0,
                                                          tm)),
                                    ctypes.byref(mll), grad, ctypes.byref(info), _stream()))
    return mll.value, [grad[i] for i in range(h.d + 2)], {
        "logdet": info.logdet, "quad": info.quad, "iterations_y": info.iterations_y,
        "iterations_probes_max": info.iterations_probes_max,
        "dquad": [info.dquad[i] for i in range(h.d + 2)], "status": st}


def batch_mll_and_grad(handles, hypers, lanczos_steps=30, tol=1e-6, maxiter=1000,
                       batch_rhs=0, batch_block=0):
    """Many problems in one persistent launch.  batch_rhs: right-hand sides
    per workgroup (2, 4 or 8), batch_block: threads per workgroup (256 or
    512); 0 = autotuned.  Returns (mll list, grad list (d+2 entries each),
    info list)."""
    L = load_library()
    n = len(handles)
    hs = (ctypes.c_void_p * n)(*[h.ptr for h in handles])
    hy = (_Hypers * n)(*[_hyp_struct(hypers[i], handles[i].d) for i in range(n)])
    mll = (ctypes.c_double * n)()
    grad = (ctypes.c_double * (5 * n))()
    infos = (_MllInfo * n)()
    st = _check(L.fkgp_batch_mll_and_grad(hs, n, hy, ctypes.byref(_MllOpts(int(lanczos_steps),
                                                                           float(tol),
                                                                           int(maxiter), 1,
                                                                           int(batch_rhs),
                                                                           int(batch_block))),
                                          mll, grad, infos, _stream()))
    return ([mll[i] for i in range(n)],
            [[grad[5 * i + k] for k in range(handles[i].d + 2)] for i in range(n)],
            [{"logdet": infos[i].logdet, "quad": infos[i].quad,
              "dquad": [infos[i].dquad[k] for k in range(handles[i].d + 2)],
              "iterations_y": infos[i].iterations_y,
              "iterations_probes_max": infos[i].iterations_probes_max,
              "batch_rhs": infos[i].batch_rhs, "batch_block": infos[i].batch_block,
              "status": st}
             for i in range(n)])


class MarginalLogLikelihood(torch.autograd.Function):
    """MLL as a differentiable function of log-hyperparameters
    theta = (log l_0..log l_{d-1}, log s, log sigma) (a 1-D CPU float64 tensor).
    Forward runs fkgp_mll_and_grad and saves the gradient; backward scales it."""

    @staticmethod
    def forward(ctx, theta, handle, lanczos_steps, tol, maxiter):
        d = handle.d
        t = theta.detach().cpu().double().tolist()
        hyp = {"lengthscale": [math.exp(v) for v in t[:d]], "outputscale": math.exp(t[d]),
               "noise": math.exp(t[d + 1])}
        val, grad, _ = mll_and_grad(handle, hyp, lanczos_steps, tol, maxiter)
        ctx.save_for_backward(torch.tensor(grad, dtype=torch.float64))
        return torch.tensor(val, dtype=torch.float64)

    @staticmethod
    def backward(ctx, gout):
        (grad,) = ctx.saved_tensors
        return gout * grad, None, None, None, None
