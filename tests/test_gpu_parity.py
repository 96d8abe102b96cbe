"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Sizes span several sort tiles and cells with a ragged tail; tolerances are the
ones the hot path is held to: FP64 statistics 1e-13 relative, FP32 statistics
1e-6, K_G products 1e-13 / 1e-6, posterior mean 1e-10 (FP64) / 1e-5 (FP32).
"""
import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2101_11751_amd")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def make_case(d, n, seed, m=None, dtype=np.float32):
    rng = np.random.default_rng(seed)
    m = m or {1: [203], 2: [37, 29], 3: [14, 11, 9]}[d]
    grid = oracle.make_grid(m, lo=0.0, hi=1.0)
    X = rng.uniform(0, 1, (d, n)).astype(dtype)
    y = (np.sin(5 * X[0].astype(np.float64)) + 0.3 * rng.standard_normal(n)).astype(dtype)
    return grid, X, y


def to_dev(X, y):
    xs = [torch.from_numpy(np.ascontiguousarray(X[k])).cuda() for k in range(X.shape[0])]
    return xs, torch.from_numpy(np.ascontiguousarray(y)).cuda()


HYP = {1: {"lengthscale": [0.05], "outputscale": 1.3, "noise": 0.2},
       2: {"lengthscale": [0.1, 0.07], "outputscale": 1.1, "noise": 0.15},
       3: {"lengthscale": [0.15, 0.2, 0.25], "outputscale": 0.9, "noise": 0.3}}


@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("stats", ["f64", "f32"])
@pytest.mark.parametrize("indt", [np.float32, np.float64])
def test_precompute_parity(d, stats, indt):
    _need_gpu()
    n = 9000 + 123 * d  # several 2048/4096-point tiles plus a ragged tail
    grid, X, y = make_case(d, n, 10 + d, dtype=indt)
    wtw_o, wty_o, yty_o = oracle.precompute(grid, X, y)
    xs, yt = to_dev(X, y)
    sdt = torch.float64 if stats == "f64" else torch.float32
    h = P.precompute(grid, xs, yt, stats_dtype=sdt)
    wtw, wty, yty = P.export_stats(h)
    tol = 1e-13 if stats == "f64" else 1e-6
    assert rel(wtw.cpu(), wtw_o) <= tol
    assert rel(wty.cpu(), wty_o) <= 1e-13
    assert abs(yty - yty_o) <= 1e-13 * abs(yty_o)
    assert h.n == n and h.m_total == int(np.prod(grid["m"]))


def test_precompute_bitwise_deterministic():
    _need_gpu()
    grid, X, y = make_case(2, 50000, 3)
    xs, yt = to_dev(X, y)
    a = P.export_stats(P.precompute(grid, xs, yt, stats_dtype=torch.float32))
    b = P.export_stats(P.precompute(grid, xs, yt, stats_dtype=torch.float32))
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]) and a[2] == b[2]


def test_precompute_empty_and_out_of_grid():
    _need_gpu()
    grid = oracle.make_grid([20, 20], lo=0.0, hi=1.0)
    e = torch.empty(0, device="cuda", dtype=torch.float32)
    h = P.precompute(grid, [e, e], e)
    wtw, wty, yty = P.export_stats(h)
    assert float(wtw.abs().sum()) == 0.0 and float(wty.abs().sum()) == 0.0 and yty == 0.0
    x0 = torch.tensor([0.5, 1.5], device="cuda")
    x1 = torch.tensor([0.5, 0.5], device="cuda")
    with pytest.raises(P.OutOfGridError):
        P.precompute(grid, [x0, x1], torch.ones(2, device="cuda"))
    x0 = torch.tensor([0.5, float("nan")], device="cuda")
    with pytest.raises(P.OutOfGridError):
        P.precompute(grid, [x0, x1], torch.ones(2, device="cuda"))
    # boundary points are interpolable
    x0 = torch.tensor([0.0, 1.0], device="cuda", dtype=torch.float64)
    x1 = torch.tensor([1.0, 0.0], device="cuda", dtype=torch.float64)
    yb = torch.ones(2, device="cuda", dtype=torch.float64)
    h = P.precompute(grid, [x0, x1], yb, stats_dtype=torch.float64)
    wtw_o, _, _ = oracle.precompute(grid, np.array([[0.0, 1.0], [1.0, 0.0]]), np.ones(2))
    assert rel(P.export_stats(h)[0].cpu(), wtw_o) <= 1e-14


@pytest.mark.parametrize("d,m", [(1, [1000]), (1, [9]), (2, [37, 29]), (2, [128, 128]),
                                 (3, [14, 11, 9]), (3, [30, 17, 6]),
                                 # four-step long lines: L = 4096, 8192, 16384; long
                                 # contiguous and long strided dimensions
                                 (1, [1500]), (1, [3000]), (1, [8192]), (2, [2100, 20]),
                                 (2, [19, 2100]), (3, [4100, 4, 5]),
                                 # L = 32768 .. 131072: spectra from the four-step FFT,
                                 # few line pairs: the three-launch passes
                                 (1, [12000]), (1, [30000]), (1, [65536]),
                                 (2, [20000, 5]), (2, [5, 20000]), (3, [17000, 4, 4]),
                                 # many long lines: one workgroup per line pair
                                 (2, [16400, 300]),
                                 # 3-D grids with 100-node inner dimensions
                                 (3, [5, 60, 100]), (3, [6, 90, 33])])
@pytest.mark.parametrize("stats", ["f64", "f32"])
def test_kg_matvec_parity(d, m, stats):
    _need_gpu()
    grid, X, y = make_case(d, 500, 7, m=m)
    xs, yt = to_dev(X, y)
    sdt = torch.float64 if stats == "f64" else torch.float32
    h = P.precompute(grid, xs, yt, stats_dtype=sdt)
    M = int(np.prod(m))
    v = np.random.default_rng(1).standard_normal((3, M))
    out = P.kg_matvec(h, HYP[d], torch.from_numpy(v).cuda()).cpu().numpy()
    ref = oracle.kg_matvec(grid, HYP[d], v)
    tol = 1e-13 if stats == "f64" else 1e-6
    for r in range(3):
        assert rel(out[r], ref[r]) <= tol


@pytest.mark.parametrize("m", [[5000], [2500, 6], [20000], [40000, 4]])
def test_solve_mean_long_lines(m):
    """Posterior mean with a grid dimension on the four-step line FFT."""
    _need_gpu()
    d = len(m)
    grid, X, y = make_case(d, 30000, 21, m=m, dtype=np.float64)
    xs, yt = to_dev(X, y)
    h = P.precompute(grid, xs, yt, stats_dtype=torch.float64)
    wtw_o, wty_o, yty_o = oracle.precompute(grid, X, y)
    hyp = {"lengthscale": [0.002] + [0.3] * (d - 1), "outputscale": 1.0, "noise": 0.2}
    mu_o, _, _ = oracle.solve_mean(grid, hyp, wtw_o, wty_o, yty_o, tol=1e-13)
    mu, info = P.solve(h, hyp, tol=1e-12, maxiter=20000)
    assert info["converged"]
    assert rel(mu.cpu(), mu_o) <= 1e-10


@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("stats", ["f64", "f32"])
def test_apply_B_parity(d, stats):
    _need_gpu()
    grid, X, y = make_case(d, 20000, 8)
    xs, yt = to_dev(X, y)
    sdt = torch.float64 if stats == "f64" else torch.float32
    h = P.precompute(grid, xs, yt, stats_dtype=sdt)
    wtw_o, _, _ = oracle.precompute(grid, X, y)
    M = h.m_total
    xv = np.random.default_rng(2).standard_normal((2, M))
    v, u = P.apply_B(h, HYP[d], torch.from_numpy(xv).cuda())
    tol = 1e-12 if stats == "f64" else 2e-6
    for r in range(2):
        vo, uo = oracle.B_apply(grid, HYP[d], wtw_o, xv[r])
        assert rel(u[r].cpu(), uo) <= tol
        assert rel(v[r].cpu(), vo) <= tol


@pytest.mark.parametrize("d", [1, 2, 3])
def test_solve_mean_fp64(d):
    _need_gpu()
    grid, X, y = make_case(d, 20000, 9, dtype=np.float64)
    xs, yt = to_dev(X, y)
    h = P.precompute(grid, xs, yt, stats_dtype=torch.float64)
    wtw_o, wty_o, yty_o = oracle.precompute(grid, X, y)
    mu_o, _, info_o = oracle.solve_mean(grid, HYP[d], wtw_o, wty_o, yty_o, tol=1e-13)
    mu, info = P.solve(h, HYP[d], tol=1e-12, maxiter=5000)
    assert info["converged"]
    assert rel(mu.cpu(), mu_o) <= 1e-10
    xq = np.random.default_rng(3).uniform(0.05, 0.95, (d, 333))
    mq = P.interpolate(h, mu, [torch.from_numpy(xq[k]).cuda() for k in range(d)])
    assert rel(mq.cpu(), oracle.interpolate(grid, mu_o, xq)) <= 1e-10


@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("op", ["f64", "stats"])
def test_solve_mean_fp32(d, op):
    """FP32 statistics; operator arithmetic FP64 (on the FP32-stored W^T W) or
    FP32 with FP64 iterative refinement: mean within 1e-5 of the oracle."""
    _need_gpu()
    grid, X, y = make_case(d, 20000, 11)
    xs, yt = to_dev(X, y)
    h = P.precompute(grid, xs, yt, stats_dtype=torch.float32)
    wtw_o, wty_o, yty_o = oracle.precompute(grid, X, y)
    mu_o, _, _ = oracle.solve_mean(grid, HYP[d], wtw_o, wty_o, yty_o, tol=1e-13)
    mu, info = P.solve(h, HYP[d], tol=1e-7, maxiter=5000, op_precision=op)
    err = rel(mu.cpu(), mu_o)
    print(f"d={d} op={op} fp32-stats mean rel err {err:.3e} iters {info['iterations']}")
    assert info["converged"]
    assert err <= 1e-5


@pytest.mark.parametrize("stats", ["f64", "f32"])
def test_solve_grid_rhs(stats):
    _need_gpu()
    grid, X, y = make_case(2, 15000, 12)
    xs, yt = to_dev(X, y)
    sdt = torch.float64 if stats == "f64" else torch.float32
    h = P.precompute(grid, xs, yt, stats_dtype=sdt)
    wtw_o, _, _ = oracle.precompute(grid, X, y)
    rhs = np.random.default_rng(4).standard_normal(h.m_total)
    ref, _ = oracle.solve_grid_rhs(grid, HYP[2], wtw_o, rhs, tol=1e-13)
    out, info = P.solve(h, HYP[2], rhs=torch.from_numpy(rhs).cuda(), tol=1e-12 if stats == "f64" else 1e-7,
                        maxiter=5000, op_precision="stats")
    assert rel(out.cpu(), ref) <= (1e-9 if stats == "f64" else 1e-4)


def test_solve_errors():
    _need_gpu()
    grid, X, y = make_case(1, 1000, 13)
    xs, yt = to_dev(X, y)
    h = P.precompute(grid, xs, yt)
    with pytest.raises(P.FkgpError):
        P.solve(h, {"lengthscale": [-1.0], "outputscale": 1.0, "noise": 0.1})
    with pytest.raises(P.FkgpError):
        P.solve(h, {"lengthscale": [0.1], "outputscale": 1.0, "noise": 0.0})
    out, info = P.solve(h, HYP[1], tol=1e-14, maxiter=2)
    assert info["status"] == P.ENOTCONV and info["iterations"] == 2


def entry_rounding_bound(grid, X, y, absx):
    """Per-row bound on |(W^T W - A) |x|| from the rounding of the entries
    themselves: any summation order of an entry sum_p w_a(p) w_b(p) errs by
    at most c eps64 (|W|^T |W|)_entry, with c the number of terms plus the
    FP64 operations of each (here 64 + the most points in a cell); the GPU
    forms entries from per-cell moments in a Bernstein basis, where every
    moment term is non-negative and every weight product has coefficients
    of one sign, so it meets the same bound."""
    wabs, _, _ = oracle.precompute(grid, X, y, absolute=True)
    d = grid["d"]
    m = list(grid["m"])
    idx = []
    for k in range(d):
        u = (X[k].astype(np.float64) - grid["origin"][k]) / grid["spacing"][k]
        idx.append(np.minimum(np.floor(u).astype(np.int64), m[k] - 3) - 1)
    counts = np.zeros([mk - 3 for mk in m])
    np.add.at(counts, tuple(idx), 1.0)
    c = 2.0 * (64 + counts.max())
    return c * 2.0 ** -52 * oracle.wtw_matvec(grid, wabs, absx)


@pytest.mark.parametrize("d,m", [(1, [1000]), (2, [37, 29]), (2, [256, 250]), (3, [14, 11, 9]),
                                 (3, [100, 20, 30]), (2, [400, 401]), (3, [60, 61, 40])])
@pytest.mark.parametrize("xdt", ["stats", "f64"])
def test_wtw_matvec_tiled_parity(d, m, xdt):
    """Banded product (windowed kernels for one and for several vectors;
    several tiles and a ragged last tile; the two largest grids hold under
    one point per cell), FP32-stored entries with FP32 or FP64 vectors."""
    _need_gpu()
    grid, X, y = make_case(d, 30000, 21, m=m)   # the larger grids: < 1 point per cell
    xs, yt = to_dev(X, y)
    h = P.precompute(grid, xs, yt, stats_dtype=torch.float32)
    wtw_o, _, _ = oracle.precompute(grid, X, y)
    v = np.random.default_rng(5).standard_normal(h.m_total)
    dt = torch.float64 if xdt == "f64" else None
    u = P.wtw_matvec(h, torch.from_numpy(v).cuda(), dt).cpu().numpy()
    # The rows are 7^d-term sums with cancellation, so the bound is the
    # standard dot-product bound n_terms * eps * (|A| |x|) per row, plus one
    # FP32 ulp of |A| |x|: the stored FP32 entries are rounded from the GPU's
    # own FP64 entries and may sit one FP32 ulp from the rounded oracle
    # values, plus the FP64 rounding of the entries (entry_rounding_bound).
    w32 = wtw_o.astype(np.float32).astype(np.float64)
    eps = 2.0 ** -52 if xdt == "f64" else 2.0 ** -23
    nt = 7 ** d

    def check(uv, vv):
        vr = vv if xdt == "f64" else vv.astype(np.float32).astype(np.float64)
        ref = oracle.wtw_matvec(grid, w32, vr)
        absax = oracle.wtw_matvec(grid, np.abs(w32), np.abs(vr))
        bound = ((2 * nt * eps + 2.0 ** -23) * absax
                 + entry_rounding_bound(grid, X, y, np.abs(vr)) + 1e-300)
        assert np.all(np.abs(uv - ref) <= bound), float(np.max(np.abs(uv - ref) / bound))

    check(u, v)
    # several vectors at once (untiled multi-vector kernel)
    V = np.random.default_rng(6).standard_normal((3, h.m_total))
    U = P.wtw_matvec(h, torch.from_numpy(V).cuda(), dt).cpu().numpy()
    for r in range(3):
        check(U[r], V[r])


@pytest.mark.parametrize("d,m", [(1, [1000]), (2, [37, 29]), (3, [14, 11, 9]),
                                 (3, [60, 61, 40])])
@pytest.mark.parametrize("stats", [torch.float32, torch.float64])
def test_wtw_matvec_dot_in_loop_form(d, m, stats):
    """The product as the CG loop launches it (u^T x reduced in the same
    launch): u equals the plain product bit for bit, u^T x its FP64 dot to
    rounding, also after repeated launches."""
    _need_gpu()
    grid, X, y = make_case(d, 20000, 23, m=m)
    xs, yt = to_dev(X, y)
    h = P.precompute(grid, xs, yt, stats_dtype=stats)
    x = torch.from_numpy(np.random.default_rng(6).standard_normal(h.m_total)).cuda()
    xp = P.padded(h, x, torch.float64)
    u_ref = torch.empty(1, h.m_total, dtype=torch.float64, device="cuda")
    P.wtw_matvec_padded(h, xp, u_ref)
    u = torch.empty_like(u_ref)
    for reps in (1, 5):
        dot = P.wtw_matvec_dot(h, xp, u, reps=reps)
        assert torch.equal(u, u_ref)
        ref = float(torch.dot(u_ref[0], x))
        absref = float(torch.dot(u_ref[0].abs(), x.abs()))
        assert abs(float(dot) - ref) <= 1e-13 * absref


def sparse_case(d, n, seed):
    """Points filling only part of the grid's box (an interval, a disk, a
    cylinder), so that whole 64-row blocks of W^T W are zero.  The region is
    a union of whole grid cells, each filled uniformly, so no node is touched
    only by a stray point in a nearly empty cell."""
    rng = np.random.default_rng(seed)
    m = {1: [1000], 2: [60, 50], 3: [30, 30, 12]}[d]
    grid = oracle.make_grid(m, lo=0.0, hi=1.0)
    nc = [mk - 3 for mk in m]                    # cells covering [0, 1]
    idx = np.stack(np.meshgrid(*[np.arange(c) for c in nc], indexing="ij"), -1).reshape(-1, d)
    ctr = (idx + 0.5) / np.asarray(nc)
    if d == 1:
        keep = ctr[:, 0] < 0.4
    else:
        keep = (ctr[:, 0] - 0.5) ** 2 + (ctr[:, 1] - 0.5) ** 2 < 0.35 ** 2
    cells = idx[keep]
    pick = cells[rng.integers(0, len(cells), n)]
    X = ((pick + rng.uniform(0, 1, (n, d))) / np.asarray(nc)).T.astype(np.float32)
    y = (np.sin(5 * X[0].astype(np.float64)) + 0.3 * rng.standard_normal(n)).astype(np.float32)
    return grid, X, y


@pytest.mark.parametrize("d", [1, 2, 3])
def test_zero_block_skipping(d):
    """The block-occupancy mask matches the stored W^T W exactly (counted on
    the host from the exported entries); the products that skip the zero
    blocks match the oracle's banded product row by row (exact zeros where
    the row is zero), and so does the solve."""
    _need_gpu()
    grid, X, y = sparse_case(d, 40000, 31 + d)
    xs, yt = to_dev(X, y)
    h = P.precompute(grid, xs, yt, stats_dtype=torch.float32)
    wtw, _, _ = P.export_stats(h)
    A = wtw.cpu().numpy()
    M, NB = A.shape
    slabs = 7 if d == 3 else 1
    nt = (M + 255) // 256
    Ap = np.zeros((nt * 256, NB), np.float32)
    Ap[:M] = A
    occ = (Ap.reshape(nt, 4, 64, slabs, NB // slabs) != 0).any(axis=(2, 4))
    assert h.wtw_blocks == nt * 4 * slabs
    assert h.wtw_block_entries == 64 * (NB // slabs)
    assert h.wtw_blocks_nonzero == int(occ.sum())
    assert 0 < h.wtw_blocks_nonzero < h.wtw_blocks
    wtw_o, wty_o, yty_o = oracle.precompute(grid, X, y)
    assert rel(A, wtw_o) <= 1e-6
    w32 = wtw_o.astype(np.float32).astype(np.float64)
    nterm = 7 ** d
    rng = np.random.default_rng(8)
    for dt, eps in ((torch.float64, 2.0 ** -52), (None, 2.0 ** -23)):
        V = rng.standard_normal((3, h.m_total))
        for k in (1, 3):   # one vector: tiled kernel; several: multi-vector kernel
            U = P.wtw_matvec(h, torch.from_numpy(V[:k]).cuda(), dt).cpu().numpy().reshape(k, -1)
            for r in range(k):
                vr = V[r] if dt is not None else V[r].astype(np.float32).astype(np.float64)
                ref = oracle.wtw_matvec(grid, w32, vr)
                absax = oracle.wtw_matvec(grid, np.abs(w32), np.abs(vr))
                # one FP32 ulp of |A||x| for the stored entries (rounded from
                # the GPU's own FP64 moments) on top of the dot-product bound
                bound = ((2 * nterm * eps + 2.0 ** -23) * absax
                         + entry_rounding_bound(grid, X, y, np.abs(vr)) + 1e-300)
                err = np.abs(U[r] - ref)
                i = int(np.argmax(err / bound))
                assert err[i] <= bound[i], (dt, k, r, i, err[i], absax[i], U[r][i], ref[i])
                assert np.all(U[r][absax == 0] == 0)
    mu_o, _, _ = oracle.solve_mean(grid, HYP[d], wtw_o, wty_o, yty_o, tol=1e-13)
    mu, info = P.solve(h, HYP[d], tol=1e-7, maxiter=5000)
    assert info["converged"]
    assert rel(mu.cpu(), mu_o) <= 1e-5


def test_solve_multi_grid_rhs():
    """k = 70 grid right-hand sides in one call (a batch of 64 and a ragged
    batch of 6): each column equals the single-right-hand-side solve and the
    oracle's factorized CG from x_0 = 0; k = 0 is a no-op."""
    _need_gpu()
    grid, X, y = make_case(2, 20000, 17, m=[30, 25], dtype=np.float64)
    xs, yt = to_dev(X, y)
    h = P.precompute(grid, xs, yt, stats_dtype=torch.float64)
    R = np.random.default_rng(4).standard_normal((70, h.m_total))
    out, info = P.solve_multi(h, HYP[2], torch.from_numpy(R).cuda(), tol=1e-12, maxiter=5000)
    assert info["converged"] and info["rel_residual"] <= 1e-12
    out = out.cpu().numpy()
    wtw_o, _, _ = oracle.precompute(grid, X, y)
    for j in (0, 37, 63, 64, 69):
        single, inf1 = P.solve(h, HYP[2], rhs=torch.from_numpy(R[j]).cuda(), tol=1e-12,
                               maxiter=5000)
        assert inf1["converged"]
        assert rel(out[j], single.cpu()) <= 1e-9
        ref, _ = oracle.solve_grid_rhs(grid, HYP[2], wtw_o, R[j], tol=1e-13)
        assert rel(out[j], ref) <= 1e-9
    empty, info0 = P.solve_multi(h, HYP[2], torch.empty(0, h.m_total, dtype=torch.float64,
                                                         device="cuda"))
    assert empty.shape[0] == 0 and info0["converged"]
