"""The host-streamed precompute: statistics from points in host memory,
sent in chunks and reduced chunk by chunk, equal the one-shot statistics up
to the order of the per-cell sums (FP64: 1e-13; FP32 storage: 1e-6) and
match the oracle; out-of-grid points are reported with their global index."""
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


def case(d, n, seed, dtype):
    rng = np.random.default_rng(seed)
    m = {1: [300], 2: [40, 33], 3: [14, 11, 9]}[d]
    grid = oracle.make_grid(m, lo=0.0, hi=1.0)
    X = rng.uniform(0, 1, (d, n)).astype(dtype)
    y = (np.sin(5 * X[0].astype(np.float64)) + 0.3 * rng.standard_normal(n)).astype(dtype)
    return grid, X, y


@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("chunk", [0, 7777, 1000])
def test_streamed_equals_one_shot(d, chunk):
    _need_gpu()
    n = 50000
    grid, X, y = case(d, n, 90 + d, np.float64)
    xs = [torch.from_numpy(np.ascontiguousarray(X[k])).cuda() for k in range(d)]
    h1 = P.precompute(grid, xs, torch.from_numpy(y).cuda(), stats_dtype=torch.float64)
    h2 = P.precompute_host(grid, [X[k] for k in range(d)], y, stats_dtype=torch.float64,
                           chunk=chunk)
    a, b = P.export_stats(h1), P.export_stats(h2)
    assert rel(b[0].cpu(), a[0].cpu()) <= 1e-13
    assert rel(b[1].cpu(), a[1].cpu()) <= 1e-13
    assert abs(b[2] - a[2]) <= 1e-13 * abs(a[2])
    assert h2.n == n and h2.wtw_blocks_nonzero == h1.wtw_blocks_nonzero
    wtw_o, wty_o, yty_o = oracle.precompute(grid, X, y)
    assert rel(b[0].cpu(), wtw_o) <= 1e-13 and rel(b[1].cpu(), wty_o) <= 1e-13


def test_streamed_fp32_storage_and_solve():
    _need_gpu()
    grid, X, y = case(2, 60000, 95, np.float32)
    h = P.precompute_host(grid, [X[0], X[1]], y, stats_dtype=torch.float32, chunk=9000)
    wtw_o, wty_o, yty_o = oracle.precompute(grid, X, y)
    wtw, wty, yty = P.export_stats(h)
    assert rel(wtw.cpu(), wtw_o) <= 1e-6 and rel(wty.cpu(), wty_o) <= 1e-13
    hyp = {"lengthscale": [0.1, 0.1], "outputscale": 1.0, "noise": 0.2}
    mu_o, _, _ = oracle.solve_mean(grid, hyp, wtw_o, wty_o, yty_o, tol=1e-13)
    mu, info = P.solve(h, hyp, tol=1e-7, maxiter=5000)
    assert info["converged"] and rel(mu.cpu(), mu_o) <= 1e-5


def test_streamed_out_of_grid_and_empty():
    _need_gpu()
    grid, X, y = case(1, 30000, 97, np.float32)
    X[0, 12345] = 5.0   # in the third chunk of 5000
    with pytest.raises(P.OutOfGridError) as e:
        P.precompute_host(grid, [X[0]], y, chunk=5000)
    assert "12345" in str(e.value)
    e0 = np.zeros(0, np.float32)
    h = P.precompute_host(grid, [e0], e0, chunk=100)
    wtw, wty, yty = P.export_stats(h)
    assert float(wtw.abs().max()) == 0.0 and yty == 0.0


@pytest.mark.parametrize("d", [1, 2, 3])
def test_streamed_probe_sketches(d):
    """Probe sketches from the streamed precompute: each point's Rademacher
    entries follow its index in the whole data set, so chunking changes
    nothing but the order of the per-cell sums (the chunk size 7,777 leaves
    cells split across chunks)."""
    _need_gpu()
    n = 40000
    grid, X, y = case(d, n, 120 + d, np.float64)
    seed, npr = 77, 5
    xs = [torch.from_numpy(np.ascontiguousarray(X[k])).cuda() for k in range(d)]
    h1 = P.precompute(grid, xs, torch.from_numpy(y).cuda(), stats_dtype=torch.float64,
                      n_probes=npr, probe_seed=seed)
    h2 = P.precompute_host(grid, [X[k] for k in range(d)], y, stats_dtype=torch.float64,
                           chunk=7777, n_probes=npr, probe_seed=seed)
    s1 = P.export_sketches(h1).cpu().numpy()
    s2 = P.export_sketches(h2).cpu().numpy()
    assert s2.shape == (npr, h1.m_total)
    assert rel(s2, s1) <= 1e-13
    sk_o = oracle.probe_sketches(grid, X, seed, npr)
    assert rel(s2, sk_o) <= 1e-13
    a, b = P.export_stats(h1), P.export_stats(h2)
    assert rel(b[1].cpu(), a[1].cpu()) <= 1e-13 and abs(b[2] - a[2]) <= 1e-13 * abs(a[2])
    # the MLL from either handle: same statistics, same probes
    hyp = {"lengthscale": [0.1] * d, "outputscale": 1.0, "noise": 0.3}
    v1, g1, _ = P.mll_and_grad(h1, hyp, 10, 1e-10, 5000)
    v2, g2, _ = P.mll_and_grad(h2, hyp, 10, 1e-10, 5000)
    assert abs(v2 - v1) <= 1e-8 * abs(v1)
    assert np.max(np.abs(np.array(g2) - np.array(g1))) <= 1e-7 * np.max(np.abs(g1))
