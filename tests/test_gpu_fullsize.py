"""Parity at the full benchmark size (3-D sweep workload, m = 100x100x30 =
300,000 grid nodes, n = 1e8 points), in the configuration bench.py times
(FP32 statistics, FP64 operator arithmetic).  The oracle cannot rebuild the
whole statistics at this size, so the checks are (a) properties that hold at
any size, (b) sampled rows of W^T W recomputed by the oracle from exactly the
points whose stencil touches the sampled node, and (c) a few solver
iterations on the full grid against the oracle running the same algorithm
from its own FP64 statistics of a smaller point set."""
import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2101_11751_amd")
W = pytest.importorskip("paper_2101_11751_amd.workloads")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_radar3d_full_precompute_properties_and_sampled_rows():
    _need_gpu()
    wl = W.radar3d(n=100_000_000, device="cuda")
    grid = wl["grid"]
    h = P.precompute(grid, wl["x"], wl["y"], stats_dtype=torch.float32)
    wtw, wty, yty = P.export_stats(h)
    n = 100_000_000
    yd = wl["y"].double()
    # properties at any size: 1^T W^T W 1 = n, sum W^T y = sum y, y^T y
    tot = float(wtw.double().sum())
    assert abs(tot - n) <= 1e-6 * n
    assert abs(float(wty.sum()) - float(yd.sum())) <= 1e-6 * float(yd.abs().sum())
    assert abs(yty - float((yd * yd).sum())) <= 1e-9 * yty
    # symmetry: (j, o) equals (j + o, -o)
    m = grid["m"]
    A = wtw.double().cpu().numpy()
    rng = np.random.default_rng(0)
    offs = np.array(np.unravel_index(np.arange(343), (7, 7, 7))).T - 3
    for j in rng.integers(0, h.m_total, 200):
        c = np.array(np.unravel_index(j, m))
        for oi in rng.integers(0, 343, 5):
            cc = c + offs[oi]
            if np.all(cc >= 0) and np.all(cc < m):
                jj = np.ravel_multi_index(tuple(cc), m)
                assert abs(A[j, oi] - A[jj, 342 - oi]) <= 1e-6 * max(abs(A[j, oi]), 1e-30) + 1e-12
    # sampled rows against the oracle on the points supporting each node
    X = torch.stack(wl["x"]).double()
    for j in (150_015, 149_000, 61_247, 222_222):
        c = np.array(np.unravel_index(j, m))
        mask = torch.ones(n, dtype=torch.bool, device="cuda")
        for k in range(3):
            u = (X[k] - grid["origin"][k]) / grid["spacing"][k]
            mask &= (u - float(c[k])).abs() < 2.0
        idx = mask.nonzero().squeeze(1)
        Xs = X[:, idx].cpu().numpy()
        ys = wl["y"][idx].double().cpu().numpy()
        wo, wyo, _ = oracle.precompute(grid, Xs, ys)
        if idx.numel() == 0:
            assert np.all(A[j] == 0)
            continue
        np.testing.assert_allclose(A[j], wo[j], rtol=0, atol=2e-6 * np.abs(wo[j]).max())
        assert abs(float(wty[j]) - wyo[j]) <= 1e-9 * np.abs(wyo).max() + 1e-9


def test_radar3d_grid_solver_iterations_match_oracle():
    """A few factorized-CG iterations on the full 300k-node grid (several
    thousand row tiles) against the oracle's iterations of the same
    algorithm."""
    _need_gpu()
    wl = W.radar3d(n=300_000, device="cuda")
    grid, hyp = wl["grid"], wl["hypers"]
    h = P.precompute(grid, wl["x"], wl["y"], stats_dtype=torch.float32)
    X = [c.double().cpu().numpy() for c in wl["x"]]
    y = wl["y"].double().cpu().numpy()
    wtw, wty, yty = oracle.precompute(grid, X, y)
    for iters in (1, 4):
        mu, info = P.solve(h, hyp, tol=1e-30, maxiter=iters)
        assert info["iterations"] == iters and not info["converged"]
        mu_o, _, info_o = oracle.solve_mean(grid, hyp, wtw, wty, yty, tol=1e-30, maxiter=iters)
        err = np.linalg.norm(mu.cpu().numpy() - mu_o) / np.linalg.norm(mu_o)
        assert err <= 1e-5, (iters, err)
