"""Marginal log-likelihood and gradient on the GPU against the oracle's
estimator with the same probes (same SplitMix64 Rademacher vectors, same
Lanczos size, tridiagonals from CG coefficients)."""
import math

import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2101_11751_amd")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def case(seed=0, m=(30, 25), n=20000, dtype=np.float32):
    rng = np.random.default_rng(seed)
    grid = oracle.make_grid(list(m), lo=0.0, hi=1.0)
    X = rng.uniform(0, 1, (2, n)).astype(dtype)
    y = (np.sin(4 * X[0].astype(np.float64)) * np.cos(3 * X[1]) + 0.2 * rng.standard_normal(n)).astype(dtype)
    hyp = {"lengthscale": [0.12, 0.09], "outputscale": 1.3, "noise": 0.25}
    return grid, X, y, hyp


def dev(X, y):
    return [torch.from_numpy(np.ascontiguousarray(X[k])).cuda() for k in range(X.shape[0])], \
        torch.from_numpy(y).cuda()


@pytest.mark.parametrize("stats", ["f64", "f32"])
@pytest.mark.parametrize("batched", [True, False])
@pytest.mark.parametrize("steps", [10, 30])
def test_mll_and_grad_parity(stats, batched, steps):
    """10 Lanczos steps: the two CG runs still agree to ~1e-12 in their
    coefficients, so the estimate is checked tightly.  30 steps: finite
    precision CG coefficients of two correct implementations drift apart
    after ~10-15 iterations (loss of orthogonality), so the tolerance is
    looser."""
    _need_gpu()
    grid, X, y, hyp = case(dtype=np.float64 if stats == "f64" else np.float32)
    N, seed = 8, 9
    xs, yt = dev(X, y)
    h = P.precompute(grid, xs, yt, stats_dtype=torch.float64 if stats == "f64" else torch.float32,
                     n_probes=N, probe_seed=seed)
    # probe sketches are bit-for-bit the same signs: compare W^T z_j
    sk = P.export_sketches(h).cpu().numpy()
    sk_o = oracle.probe_sketches(grid, X, seed, N)
    np.testing.assert_allclose(sk, sk_o, rtol=0, atol=1e-11 * np.abs(sk_o).max())
    wtw, wty, yty = oracle.precompute(grid, X, y)
    mll_o, g_o, inf_o = oracle.mll_and_grad(grid, hyp, wtw, wty, yty, X.shape[1], sk_o,
                                            lanczos_steps=steps, tol=1e-10)
    mll, g, inf = P.mll_and_grad(h, hyp, lanczos_steps=steps, tol=1e-10, maxiter=3000,
                                 batched=batched)
    if stats == "f64":
        tol_m, tol_g = (1e-10, 1e-7) if steps == 10 else (1e-6, 1e-5)
    else:
        tol_m, tol_g = (1e-6, 1e-4) if steps == 10 else (1e-6, 1e-4)
    print(f"stats={stats} batched={batched} steps={steps}: mll {mll:.12g} vs {mll_o:.12g}; "
          f"grad {np.array(g)} vs {g_o}")
    # q = y^T A^{-1} y from two solves stopped at relative residual 1e-10:
    # |y^T A^{-1} r| <= ||y||^2 tol / sigma^2 each (lambda_min(A) >= sigma^2)
    s2 = hyp["noise"] ** 2
    q_bound = 2 * 1e-10 * float(np.dot(y.astype(np.float64), y)) / s2
    # the MLL is a small difference of large terms: scale by their magnitude
    scale = abs(inf_o["logdet"]) + abs(inf_o["q"]) + X.shape[1] * math.log(2 * math.pi)
    assert abs(mll - mll_o) <= tol_m * scale + 0.5 * q_bound, (mll, mll_o)
    assert abs(inf["logdet"] - inf_o["logdet"]) <= tol_m * abs(inf_o["logdet"])
    assert abs(inf["quad"] - inf_o["q"]) <= tol_m * abs(inf_o["q"]) + q_bound
    np.testing.assert_allclose(g, g_o, rtol=0, atol=tol_g * np.abs(g_o).max())


def test_mll_logdet_within_standard_errors_of_exact():
    """With 31 probes the GPU's SLQ log-determinant lies within 4 standard
    errors (estimated from the same probes' samples) of the exact dense
    log-determinant, and the Hutchinson gradient is close to the exact
    dense gradient."""
    _need_gpu()
    grid, X, y, hyp = case(1, m=(14, 12), n=3000, dtype=np.float64)
    xs, yt = dev(X, y)
    h = P.precompute(grid, xs, yt, stats_dtype=torch.float64, n_probes=31, probe_seed=3)
    mll, g, inf = P.mll_and_grad(h, hyp, lanczos_steps=60, tol=1e-11, maxiter=3000)
    W = oracle.dense_w(grid, X)
    A = W @ oracle.kg_dense(grid, hyp) @ W.T + hyp["noise"] ** 2 * np.eye(X.shape[1])
    exact = np.linalg.slogdet(A)[1]
    wtw, wty, yty = oracle.precompute(grid, X, y)
    sk = oracle.probe_sketches(grid, X, 3, 31)
    _, _, inf_o = oracle.mll_and_grad(grid, hyp, wtw, wty, yty, X.shape[1], sk,
                                      lanczos_steps=60, tol=1e-11)
    smp = inf_o["logdet_samples"]
    se = smp.std(ddof=1) / np.sqrt(len(smp))
    assert abs(inf["logdet"] - exact) <= 4 * se + 1e-8 * abs(exact), (inf["logdet"], exact, se)
    g_exact = oracle.ski_dense_grad(grid, hyp, X, y)
    assert np.all(np.abs(np.array(g) - g_exact) <= 0.3 * np.abs(g_exact) + 3.0), (g, g_exact)


def test_autograd_function():
    _need_gpu()
    grid, X, y, hyp = case(2, m=(20, 18), n=8000)
    xs, yt = dev(X, y)
    h = P.precompute(grid, xs, yt, n_probes=4, probe_seed=1)
    theta = torch.tensor([math.log(0.12), math.log(0.09), math.log(1.3), math.log(0.25)],
                         dtype=torch.float64, requires_grad=True)
    val = P.MarginalLogLikelihood.apply(theta, h, 30, 1e-8, 2000)
    (2.0 * val).backward()
    t = [math.exp(v) for v in theta.detach().tolist()]
    hyp_t = {"lengthscale": t[:2], "outputscale": t[2], "noise": t[3]}
    mll, g, _ = P.mll_and_grad(h, hyp_t, 30, 1e-8, 2000)
    # deterministic reductions: the same inputs give bit-identical results
    assert float(val) == mll
    np.testing.assert_array_equal(theta.grad.numpy(), 2.0 * np.array(g))


def test_mll_errors():
    _need_gpu()
    grid, X, y, hyp = case(3, n=500)
    xs, yt = dev(X, y)
    h = P.precompute(grid, xs, yt)
    with pytest.raises(P.FkgpError):
        P.mll_and_grad(h, hyp)
    with pytest.raises(P.FkgpError):   # at most 31 probes
        P.precompute(oracle.make_grid([10, 10, 10], lo=0.0, hi=1.0),
                     [xs[0], xs[1], xs[0]], yt, n_probes=32)


def test_mll_exact_trace_gradient():
    """trace="exact": the traces tr(A^{-1} dA) come from S = W^T A^{-1} W
    (one grid solve per node: 120 nodes, batches of 64 and 56), so the
    gradient is deterministic: it equals the oracle's exact-trace gradient
    and central differences of the oracle's dense Def. 2 MLL."""
    _need_gpu()
    grid, X, y, hyp = case(seed=4, m=(12, 10), n=1500, dtype=np.float64)
    N, seed = 4, 5
    xs, yt = dev(X, y)
    h = P.precompute(grid, xs, yt, stats_dtype=torch.float64, n_probes=N, probe_seed=seed)
    mll, g, inf = P.mll_and_grad(h, hyp, lanczos_steps=10, tol=1e-12, maxiter=5000,
                                 trace="exact")
    wtw, wty, yty = oracle.precompute(grid, X, y)
    sk_o = oracle.probe_sketches(grid, X, seed, N)
    _, g_o, _ = oracle.mll_and_grad(grid, hyp, wtw, wty, yty, X.shape[1], sk_o,
                                    lanczos_steps=10, tol=1e-13, exact_trace=True)
    np.testing.assert_allclose(g, g_o, rtol=0, atol=1e-7 * np.abs(g_o).max())
    # central differences of the dense exact MLL in (log l_k, log s, log sigma)
    eps = 1e-4
    fd = []
    for i in range(len(g)):
        vals = []
        for sgn in (1, -1):
            hp = {"lengthscale": list(hyp["lengthscale"]), "outputscale": hyp["outputscale"],
                  "noise": hyp["noise"]}
            f = math.exp(sgn * eps)
            if i < 2:
                hp["lengthscale"][i] *= f
            elif i == 2:
                hp["outputscale"] *= f
            else:
                hp["noise"] *= f
            vals.append(oracle.ski_dense_mll(grid, hp, X, y))
        fd.append((vals[0] - vals[1]) / (2 * eps))
    np.testing.assert_allclose(g, fd, rtol=0, atol=1e-5 * np.abs(fd).max())
    # exact traces need one solve per node: refused above 4096 nodes
    g2, X2, y2, hyp2 = case(seed=5, m=(70, 60), n=2000, dtype=np.float64)
    h2 = P.precompute(g2, *dev(X2, y2), stats_dtype=torch.float64, n_probes=2, probe_seed=1)
    with pytest.raises(P.FkgpError, match="4096"):
        P.mll_and_grad(h2, hyp2, trace="exact")


def test_mll_long_1d_lines_fft_spectra():
    """1-D grid of 3000 nodes (circulant of 8192 points, four-step passes,
    spectra and derivative spectra from the forward four-step FFT): MLL and
    gradient against the oracle's estimator with the same probes."""
    _need_gpu()
    rng = np.random.default_rng(12)
    grid = oracle.make_grid([3000], lo=0.0, hi=1.0)
    X = rng.uniform(0, 1, (1, 30000))
    y = np.sin(9 * X[0]) + 0.2 * rng.standard_normal(30000)
    hyp = {"lengthscale": [0.01], "outputscale": 1.1, "noise": 0.2}
    N, seed = 4, 21
    h = P.precompute(grid, [torch.from_numpy(X[0]).cuda()], torch.from_numpy(y).cuda(),
                     stats_dtype=torch.float64, n_probes=N, probe_seed=seed)
    mll, g, inf = P.mll_and_grad(h, hyp, lanczos_steps=10, tol=1e-10, maxiter=5000)
    wtw, wty, yty = oracle.precompute(grid, X, y)
    sk = oracle.probe_sketches(grid, X, seed, N)
    mll_o, g_o, inf_o = oracle.mll_and_grad(grid, hyp, wtw, wty, yty, X.shape[1], sk,
                                            lanczos_steps=10, tol=1e-10)
    s2 = hyp["noise"] ** 2
    q_bound = 2 * 1e-10 * float(np.dot(y, y)) / s2
    scale = abs(inf_o["logdet"]) + abs(inf_o["q"]) + X.shape[1] * math.log(2 * math.pi)
    assert abs(mll - mll_o) <= 1e-10 * scale + 0.5 * q_bound, (mll, mll_o)
    np.testing.assert_allclose(g, g_o, rtol=0, atol=1e-7 * np.abs(g_o).max())


@pytest.mark.parametrize("indt", [np.float32, np.float64])
def test_mll_3d_probe_sketches(indt):
    """3-D handles with probe sketches (the sort carries each point's index
    in the slot of y, which the moments read back by index): sketches, W^T y,
    W^T W and the MLL with its gradient against the oracle."""
    _need_gpu()
    rng = np.random.default_rng(33)
    grid = oracle.make_grid([10, 9, 8], lo=0.0, hi=1.0)
    n = 20000
    X = rng.uniform(0, 1, (3, n)).astype(indt)
    y = (np.sin(3 * X[0].astype(np.float64)) * X[1] + 0.2 * rng.standard_normal(n)).astype(indt)
    hyp = {"lengthscale": [0.3, 0.25, 0.35], "outputscale": 1.1, "noise": 0.3}
    N, seed = 31, 17
    xs = [torch.from_numpy(np.ascontiguousarray(X[k])).cuda() for k in range(3)]
    h = P.precompute(grid, xs, torch.from_numpy(y).cuda(), stats_dtype=torch.float64,
                     n_probes=N, probe_seed=seed)
    sk = P.export_sketches(h).cpu().numpy()
    sk_o = oracle.probe_sketches(grid, X, seed, N)
    np.testing.assert_allclose(sk, sk_o, rtol=0, atol=1e-11 * np.abs(sk_o).max())
    wtw, wty, yty = P.export_stats(h)
    wtw_o, wty_o, yty_o = oracle.precompute(grid, X, y)
    assert np.linalg.norm(wtw.cpu().numpy() - wtw_o) <= 1e-13 * np.linalg.norm(wtw_o)
    assert np.linalg.norm(wty.cpu().numpy() - wty_o) <= 1e-13 * np.linalg.norm(wty_o)
    assert abs(yty - yty_o) <= 1e-13 * yty_o
    mll, g, inf = P.mll_and_grad(h, hyp, lanczos_steps=10, tol=1e-10, maxiter=3000)
    mll_o, g_o, inf_o = oracle.mll_and_grad(grid, hyp, wtw_o, wty_o, yty_o, n, sk_o,
                                            lanczos_steps=10, tol=1e-10)
    yd = y.astype(np.float64)
    q_bound = 2 * 1e-10 * float(yd @ yd) / hyp["noise"] ** 2
    scale = abs(inf_o["logdet"]) + abs(inf_o["q"]) + n * math.log(2 * math.pi)
    assert abs(mll - mll_o) <= 1e-10 * scale + 0.5 * q_bound, (mll, mll_o)
    np.testing.assert_allclose(g, g_o, rtol=0, atol=1e-7 * np.abs(g_o).max())
