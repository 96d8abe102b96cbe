"""The plain SKI baseline (CG in n-space on W K_G W^T + s2 I, the iteration
the factorized CG replaces; Sec. 2.3): its posterior-mean grid weights match
the oracle's dense Def. 2 solve on small inputs, and the factorized solve and
the oracle's factorized CG on larger ones (Theorem 1 / Fact 2: both forms give
the same weights)."""
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


HYP = {1: {"lengthscale": [0.08], "outputscale": 1.2, "noise": 0.2},
       2: {"lengthscale": [0.15, 0.12], "outputscale": 0.9, "noise": 0.25},
       3: {"lengthscale": [0.3, 0.25, 0.35], "outputscale": 1.1, "noise": 0.3}}


def case(d, n, m, seed, dtype):
    rng = np.random.default_rng(seed)
    grid = oracle.make_grid(m, lo=0.0, hi=1.0)
    X = rng.uniform(0, 1, (d, n)).astype(dtype)
    y = (np.sin(6 * X[0].astype(np.float64)) + 0.3 * rng.standard_normal(n)).astype(dtype)
    xs = [torch.from_numpy(np.ascontiguousarray(X[k])).cuda() for k in range(d)]
    return grid, X, y, xs, torch.from_numpy(y).cuda()


@pytest.mark.parametrize("d,n,m", [(1, 1500, [60]), (2, 1200, [12, 10]), (3, 900, [8, 7, 6])])
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_ski_solve_matches_dense_def2(d, n, m, dtype):
    _need_gpu()
    grid, X, y, xs, yt = case(d, n, m, 40 + d, dtype)
    h = P.precompute(grid, xs, yt, stats_dtype=torch.float64, keep_points=True)
    mu, info = P.ski_solve(h, HYP[d], tol=1e-12, maxiter=5000)
    assert info["converged"] and info["iterations"] > 1
    mu_o, _, _ = oracle.ski_dense_mean(grid, HYP[d], X.astype(np.float64), y.astype(np.float64))
    assert rel(mu.cpu(), mu_o) <= 1e-8


@pytest.mark.parametrize("d,m", [(1, [800]), (2, [40, 33]), (3, [14, 12, 10])])
def test_ski_solve_matches_factorized(d, m):
    _need_gpu()
    grid, X, y, xs, yt = case(d, 30000, m, 50 + d, np.float32)
    h = P.precompute(grid, xs, yt, stats_dtype=torch.float64, keep_points=True)
    mu_s, info_s = P.ski_solve(h, HYP[d], tol=1e-11, maxiter=20000)
    mu_g, info_g = P.solve(h, HYP[d], tol=1e-11, maxiter=20000)
    assert info_s["converged"] and info_g["converged"]
    wtw_o, wty_o, yty_o = oracle.precompute(grid, X, y)
    mu_o, _, _ = oracle.solve_mean(grid, HYP[d], wtw_o, wty_o, yty_o, tol=1e-13)
    assert rel(mu_s.cpu(), mu_o) <= 1e-7
    assert rel(mu_s.cpu(), mu_g.cpu()) <= 1e-7


def test_ski_solve_errors_and_empty():
    _need_gpu()
    grid, X, y, xs, yt = case(1, 500, [50], 7, np.float32)
    h = P.precompute(grid, xs, yt)
    with pytest.raises(P.FkgpError):
        P.ski_solve(h, HYP[1])
    e = torch.empty(0, device="cuda", dtype=torch.float32)
    h0 = P.precompute(grid, [e], e, keep_points=True)
    mu, info = P.ski_solve(h0, HYP[1])
    assert info["converged"] and float(mu.abs().max()) == 0.0


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_kept_points_with_probe_sketches_3d(dtype):
    """In 3-D the sort carries the point index in y's slot when probe sketches
    are requested; the kept points get y back from the input, so one handle
    serves the plain SKI solve and the MLL: its SKI mean, statistics and
    sketches equal those of handles made with either option alone."""
    _need_gpu()
    d, m = 3, [14, 12, 10]
    grid, X, y, xs, yt = case(d, 20000, m, 61, dtype)
    hb = P.precompute(grid, xs, yt, stats_dtype=torch.float64, keep_points=True, n_probes=4,
                      probe_seed=9)
    hk = P.precompute(grid, xs, yt, stats_dtype=torch.float64, keep_points=True)
    hp = P.precompute(grid, xs, yt, stats_dtype=torch.float64, n_probes=4, probe_seed=9)
    mu_b, ib = P.ski_solve(hb, HYP[d], tol=1e-11, maxiter=20000)
    mu_k, ik = P.ski_solve(hk, HYP[d], tol=1e-11, maxiter=20000)
    assert ib["converged"] and ik["converged"]
    assert torch.equal(mu_b, mu_k)   # same kept points, same arithmetic
    a, b = P.export_stats(hb), P.export_stats(hp)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]) and a[2] == b[2]
    assert torch.equal(P.export_sketches(hb), P.export_sketches(hp))
