"""Posterior covariance between query points (the covariance expression of
SKI inference, Def. 2): the device result matches the oracle's dense
Cholesky form on small inputs, Fact 2's grid form sigma^2 (K_G W^T W +
sigma^2 I)^{-1} K_G on larger ones, and the prior Wq K_G Wq^T when there are
no data."""
import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2101_11751_amd")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


HYP = {1: {"lengthscale": [0.08], "outputscale": 1.2, "noise": 0.2},
       2: {"lengthscale": [0.15, 0.12], "outputscale": 0.9, "noise": 0.25},
       3: {"lengthscale": [0.3, 0.25, 0.35], "outputscale": 1.1, "noise": 0.3}}


def case(d, n, m, seed, dtype=np.float64, nq=12):
    rng = np.random.default_rng(seed)
    grid = oracle.make_grid(m, lo=0.0, hi=1.0)
    X = rng.uniform(0, 1, (d, n)).astype(dtype)
    y = (np.sin(6 * X[0].astype(np.float64)) + 0.3 * rng.standard_normal(n)).astype(dtype)
    Xq = rng.uniform(0, 1, (d, nq)).astype(dtype)
    xs = [torch.from_numpy(np.ascontiguousarray(X[k])).cuda() for k in range(d)]
    xq = [torch.from_numpy(np.ascontiguousarray(Xq[k])).cuda() for k in range(d)]
    return grid, X, y, Xq, xs, torch.from_numpy(y).cuda(), xq


def fact2_cov(grid, hyp, X, Xq):
    """Wq C Wq^T with C = sigma^2 (K_G W^T W + sigma^2 I)^{-1} K_G (Fact 2)."""
    wtw, _, _ = oracle.precompute(grid, X, np.zeros(X.shape[1]))
    A = oracle.wtw_dense_from_dia(grid, wtw)
    KG = oracle.kg_dense(grid, hyp)
    s2 = hyp["noise"] ** 2
    C = s2 * np.linalg.solve(KG @ A + s2 * np.eye(A.shape[0]), KG)
    Wq = oracle.dense_w(grid, Xq)
    return Wq @ C @ Wq.T


@pytest.mark.parametrize("d,n,m", [(1, 500, [60]), (2, 400, [12, 10]), (3, 300, [8, 7, 6])])
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_cov_matches_dense_def2(d, n, m, dtype):
    _need_gpu()
    grid, X, y, Xq, xs, yt, xq = case(d, n, m, 90 + d, dtype)
    h = P.precompute(grid, xs, yt, stats_dtype=torch.float64)
    C, info = P.posterior_cov(h, HYP[d], xq, tol=1e-13, maxiter=5000)
    assert info["converged"] and info["iterations"] > 1
    ref = oracle.ski_dense_cov(grid, HYP[d], X.astype(np.float64), Xq.astype(np.float64))
    C = C.cpu().numpy()
    scale = np.abs(np.diag(ref)).max()
    assert np.abs(C - ref).max() <= 1e-8 * scale
    assert np.array_equal(C, C.T)


@pytest.mark.parametrize("kernel", ["se", "matern32"])
def test_cov_many_queries_fact2(kernel):
    """100 query points: two batches of right-hand sides (64 + 36) and a 2 x 2
    tiling of the pair matrix with ragged edges; n = 30000 points."""
    _need_gpu()
    grid, X, y, Xq, xs, yt, xq = case(2, 30000, [40, 33], 7, np.float32, nq=100)
    hyp = dict(HYP[2], kernel=kernel)
    h = P.precompute(grid, xs, yt, stats_dtype=torch.float64)
    C, info = P.posterior_cov(h, hyp, xq, tol=1e-12, maxiter=20000)
    assert info["converged"] and info["rel_residual"] <= 1e-12
    ref = fact2_cov(grid, hyp, X.astype(np.float64), Xq.astype(np.float64))
    C = C.cpu().numpy()
    scale = np.abs(np.diag(ref)).max()
    assert np.abs(C - ref).max() <= 1e-7 * scale
    assert np.linalg.eigvalsh(C).min() > -1e-9 * scale


def test_cov_fp32_stats():
    """W^T W stored in FP32 (entries upcast exactly, FP64 arithmetic): the
    result differs from the FP64 oracle only through the storage rounding."""
    _need_gpu()
    grid, X, y, Xq, xs, yt, xq = case(1, 20000, [300], 11, np.float32, nq=20)
    h = P.precompute(grid, xs, yt, stats_dtype=torch.float32)
    C, info = P.posterior_cov(h, HYP[1], xq, tol=1e-12, maxiter=20000)
    assert info["converged"]
    ref = fact2_cov(grid, HYP[1], X.astype(np.float64), Xq.astype(np.float64))
    scale = np.abs(np.diag(ref)).max()
    assert np.abs(C.cpu().numpy() - ref).max() <= 1e-4 * scale


def test_cov_no_data_is_prior():
    """n = 0: W^T W = 0, every right-hand side is zero and the result is the
    prior covariance Wq K_G Wq^T."""
    _need_gpu()
    grid = oracle.make_grid([20, 16], lo=0.0, hi=1.0)
    e = torch.empty(0, device="cuda", dtype=torch.float64)
    h = P.precompute(grid, [e, e], e, stats_dtype=torch.float64)
    Xq = np.random.default_rng(3).uniform(0, 1, (2, 9))
    xq = [torch.from_numpy(np.ascontiguousarray(Xq[k])).cuda() for k in range(2)]
    C, info = P.posterior_cov(h, HYP[2], xq)
    assert info["converged"] and info["iterations"] == 0
    Wq = oracle.dense_w(grid, Xq)
    ref = Wq @ oracle.kg_dense(grid, HYP[2]) @ Wq.T
    np.testing.assert_allclose(C.cpu().numpy(), ref, rtol=0, atol=1e-13 * np.abs(ref).max())


def test_cov_single_query_and_errors():
    _need_gpu()
    grid, X, y, Xq, xs, yt, xq = case(1, 500, [60], 5, np.float64, nq=1)
    h = P.precompute(grid, xs, yt, stats_dtype=torch.float64)
    C, info = P.posterior_cov(h, HYP[1], xq, tol=1e-13)
    ref = oracle.ski_dense_cov(grid, HYP[1], X, Xq)
    assert C.shape == (1, 1)
    assert abs(float(C[0, 0]) - ref[0, 0]) <= 1e-8 * abs(ref[0, 0])
    with pytest.raises(P.OutOfGridError):
        P.posterior_cov(h, HYP[1], [torch.tensor([0.5, 7.0], device="cuda", dtype=torch.float64)])
    with pytest.raises(P.FkgpError):
        P.posterior_cov(h, HYP[1], [torch.empty(0, device="cuda", dtype=torch.float64)])
    with pytest.raises(P.FkgpError):
        P.posterior_cov(h, HYP[1], [torch.full((4097,), 0.5, device="cuda",
                                                dtype=torch.float64)])


def test_cov_dense_data_small_posterior():
    """Many points per cell (n = 30000 on 300 nodes, sigma = 0.1): the
    posterior variances are ~1e-3 of the prior's, so the reduction term must
    be accurate far below the prior's size.  Grid right-hand sides keep the
    residual in the form W r_hat (no cancelling terms in ||r||), so the
    solves reach tol = 1e-12 and the result matches Fact 2's grid form."""
    _need_gpu()
    rng = np.random.default_rng(21)
    grid = oracle.make_grid([300], lo=0.0, hi=1.0)
    X = rng.uniform(0, 1, (1, 30000))
    y = np.sin(6 * X[0]) + 0.1 * rng.standard_normal(30000)
    Xq = rng.uniform(0, 1, (1, 40))
    hyp = {"lengthscale": [0.08], "outputscale": 1.0, "noise": 0.1}
    h = P.precompute(grid, [torch.from_numpy(X[0]).cuda()], torch.from_numpy(y).cuda(),
                     stats_dtype=torch.float64)
    C, info = P.posterior_cov(h, hyp, [torch.from_numpy(Xq[0]).cuda()], tol=1e-12,
                              maxiter=20000)
    assert info["converged"], info
    ref = fact2_cov(grid, hyp, X, Xq)
    scale = np.abs(np.diag(ref)).max()
    err = np.abs(C.cpu().numpy() - ref).max()
    print(f"posterior scale {scale:.3e}, max error {err:.3e}, iterations {info['iterations']}")
    assert err <= 1e-6 * scale
    c = P.love_build(h, hyp, 300)
    errk = np.abs(c.cov([torch.from_numpy(Xq[0]).cuda()]).cpu().numpy() - ref).max()
    print(f"rank {c.rank}: max error {errk:.3e}")
    assert errk <= 1e-6 * scale


def test_cov_maximum_query_count_sampled():
    """nq = 4096 (the largest call): 64 batches of right-hand sides and a
    64 x 64 tiling of the pair matrix; sampled rows and columns against Fact
    2's grid form, symmetry, and the rank-k covariance on the same points."""
    _need_gpu()
    rng = np.random.default_rng(31)
    grid = oracle.make_grid([40, 30], lo=0.0, hi=1.0)
    X = rng.uniform(0, 1, (2, 20000))
    y = np.sin(5 * X[0]) + 0.2 * rng.standard_normal(20000)
    Xq = rng.uniform(0, 1, (2, 4096))
    hyp = {"lengthscale": [0.15, 0.12], "outputscale": 0.9, "noise": 0.25}
    xs = [torch.from_numpy(X[k]).cuda() for k in range(2)]
    xq = [torch.from_numpy(Xq[k]).cuda() for k in range(2)]
    h = P.precompute(grid, xs, torch.from_numpy(y).cuda(), stats_dtype=torch.float64)
    C, info = P.posterior_cov(h, hyp, xq, tol=1e-12, maxiter=20000)
    assert info["converged"]
    C = C.cpu().numpy()
    assert np.array_equal(C, C.T)
    idx = np.concatenate([np.arange(5), rng.choice(4096, 20, replace=False), [4095]])
    ref = fact2_cov(grid, hyp, X, Xq[:, idx])
    scale = np.abs(np.diag(ref)).max()
    assert np.abs(C[np.ix_(idx, idx)] - ref).max() <= 1e-7 * scale
    c = P.love_build(h, hyp, 120)
    Ck = c.cov(xq).cpu().numpy()
    wtw, wty, yty = oracle.precompute(grid, X, y)
    ref_k = oracle.love_cov(grid, hyp, wtw, wty, yty, Xq[:, idx], c.rank)
    assert np.abs(Ck[np.ix_(idx, idx)] - ref_k).max() <= 1e-8 * np.abs(np.diag(ref_k)).max()
