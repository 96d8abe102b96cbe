"""Pins of the oracle against what the paper and the mathematics fix
(CPU only).  Each test would fail on a plausible slip in the oracle: a wrong
weight coefficient, a transposed offset, a dropped sigma^2, a wrong sign or
index in the factorized recurrences."""
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg as sla

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def keys_kernel(s):
    """Textbook Keys kernel (a = -1/2), independent of the oracle's
    polynomial-in-t form."""
    s = np.abs(s)
    return np.where(s <= 1, 1.5 * s ** 3 - 2.5 * s ** 2 + 1,
                    np.where(s < 2, -0.5 * s ** 3 + 2.5 * s ** 2 - 4 * s + 2, 0.0))


def hat_kernel(s):
    """Linear-interpolation basis function max(0, 1 - |s|)."""
    return np.maximum(0.0, 1.0 - np.abs(s))


def dense_w_textbook(grid, X):
    """W[i, j] = prod_k phi(u_ik - j_k) over all grid nodes (brute force),
    phi the Keys kernel, or the hat function for linear interpolation."""
    d = grid["d"]
    m = grid["m"]
    n = X.shape[1]
    M = int(np.prod(m))
    phi = hat_kernel if grid.get("interp", "cubic") == "linear" else keys_kernel
    coords = np.array(np.unravel_index(np.arange(M), m))  # [d, M]
    W = np.ones((n, M))
    for k in range(d):
        u = (X[k] - grid["origin"][k]) / grid["spacing"][k]
        W *= phi(u[:, None] - coords[k][None, :])
    return W


def rand_points(rng, grid, n):
    X = []
    for k in range(grid["d"]):
        lo = grid["origin"][k] + grid["spacing"][k]
        hi = grid["origin"][k] + (grid["m"][k] - 2) * grid["spacing"][k]
        X.append(rng.uniform(lo, hi, n))
    return np.array(X)


# --------------------------------------------------------------------------
# Interpolation weights (Keys cubic convolution, Sec. 3 / Fig. 1 basis).
# --------------------------------------------------------------------------
def test_keys_weights_golden():
    rows = np.loadtxt(os.path.join(GOLD, "keys_weights.txt"))
    grid = oracle.make_grid([10], origin=[0.0], spacing=[1.0])
    for t, *w in rows:
        _, wts, _ = oracle.stencils(grid, np.array([4.0 + t]))
        # t = 1 is assigned to cell 4 with t = 0 (floor); compare by node
        nodes, _, _ = oracle.stencils(grid, np.array([4.0 + t]))
        full = np.zeros(10)
        full[nodes[0]] = wts[0]
        ref = np.zeros(10)
        ref[3:7] = w
        np.testing.assert_allclose(full, ref, atol=1e-15)


def test_keys_weights_polynomial_reproduction():
    grid = oracle.make_grid([20], origin=[0.0], spacing=[1.0])
    u = np.linspace(1.0, 18.0, 997)
    nodes, w, _ = oracle.stencils(grid, u)
    np.testing.assert_allclose(w.sum(1), 1.0, atol=1e-14)
    np.testing.assert_allclose((w * nodes).sum(1), u, atol=1e-12)
    np.testing.assert_allclose((w * nodes ** 2).sum(1), u ** 2, atol=1e-10)
    # cubic is not reproduced (third-order kernel)
    assert np.max(np.abs((w * nodes ** 3).sum(1) - u ** 3)) > 1e-3


def test_keys_weights_match_textbook_kernel_and_continuity():
    rng = np.random.default_rng(0)
    grid = oracle.make_grid([12, 9], origin=[-0.3, 1.0], spacing=[0.1, 0.25])
    X = rand_points(rng, grid, 300)
    # include exact node positions and the upper boundary u = m - 2
    X[:, 0] = [grid["origin"][0] + 5 * grid["spacing"][0], grid["origin"][1] + 7 * grid["spacing"][1]]
    X[:, 1] = [grid["origin"][0] + 10 * grid["spacing"][0], grid["origin"][1] + 1 * grid["spacing"][1]]
    W = oracle.dense_w(grid, X)
    Wt = dense_w_textbook(grid, X)
    np.testing.assert_allclose(W, Wt, atol=1e-14)


def _keys_exact(s):
    """Textbook Keys kernel (a = -1/2) in exact rational arithmetic."""
    s = abs(s)
    if s <= 1:
        return Fraction(3, 2) * s ** 3 - Fraction(5, 2) * s ** 2 + 1
    if s < 2:
        return -Fraction(1, 2) * s ** 3 + Fraction(5, 2) * s ** 2 - 4 * s + 2
    return Fraction(0)


def test_keys_weights_relative_accuracy_against_exact_rationals():
    """Each weight to a few units in its own last place, also where it is
    tiny (t or 1 - t near 0), against the kernel evaluated exactly at the
    same (binary) offset."""
    grid = oracle.make_grid([10], origin=[0.0], spacing=[1.0])
    ts = [2.0 ** -k for k in range(1, 40, 3)] + [1 - 2.0 ** -k for k in range(1, 40, 3)]
    ts += list(np.random.default_rng(9).uniform(0, 1, 200))
    for t in ts:
        nodes, w, _ = oracle.stencils(grid, np.array([4.0 + t]))
        u = Fraction(4.0 + t)
        for a in range(4):
            ex = _keys_exact(u - int(nodes[0, a]))
            assert abs(Fraction(float(w[0, a])) - ex) <= 8 * Fraction(2) ** -53 * abs(ex), (t, a)


@pytest.mark.parametrize("m,n", [([300], 300), ([18, 17], 300)])
def test_wtw_entries_against_exact_rationals_one_point_per_cell(m, n):
    """About one point per cell, so many entries are single products of
    small weights: every entry within 64 units of 2^-53 times the matching
    entry of |W|^T |W| of the exact sum (weights and products in rationals)."""
    rng = np.random.default_rng(5)
    grid = oracle.make_grid(m, lo=0.0, hi=1.0)
    d = len(m)
    X = rng.uniform(0, 1, (d, n))
    wtw, _, _ = oracle.precompute(grid, X, np.ones(n))
    M = int(np.prod(m))
    ex = np.zeros((M, 7 ** d), object)
    ex[:] = Fraction(0)
    exa = np.zeros((M, 7 ** d))
    g0, h = grid["origin"], grid["spacing"]
    for i in range(n):
        base, w1 = [], []
        for k in range(d):
            u = (X[k, i] - g0[k]) / h[k]
            b = min(int(np.floor(u)), m[k] - 3)
            uf = Fraction(u)
            base.append(b)
            w1.append([_keys_exact(uf - (b - 1 + a)) for a in range(4)])
        for sa in np.ndindex(*([4] * d)):
            for sb in np.ndindex(*([4] * d)):
                wa = wb = Fraction(1)
                for k in range(d):
                    wa *= w1[k][sa[k]]
                    wb *= w1[k][sb[k]]
                ja = np.ravel_multi_index([base[k] - 1 + sa[k] for k in range(d)], m)
                o = np.ravel_multi_index([sb[k] - sa[k] + 3 for k in range(d)], [7] * d)
                ex[ja, o] += wa * wb
                exa[ja, o] += abs(float(wa * wb))
    exf = np.vectorize(float)(ex)
    assert np.all(np.abs(wtw - exf) <= 64 * 2.0 ** -53 * exa)


def test_out_of_grid_rejected():
    grid = oracle.make_grid([10], origin=[0.0], spacing=[1.0])
    for bad in (0.999, 8.0001, np.nan):
        with pytest.raises(ValueError):
            oracle.precompute(grid, np.array([3.0, bad]), np.array([1.0, 1.0]))
    oracle.precompute(grid, np.array([1.0, 8.0]), np.array([1.0, 1.0]))


# --------------------------------------------------------------------------
# Sufficient statistics (Sec. 3.1; Claim 2).
# --------------------------------------------------------------------------
@pytest.mark.parametrize("m", [[11], [7, 9], [6, 5, 7]])
def test_wtw_bruteforce_dense(m):
    rng = np.random.default_rng(len(m))
    grid = oracle.make_grid(m, origin=[0.5] * len(m), spacing=[0.3] * len(m))
    n = 400
    X = rand_points(rng, grid, n)
    y = rng.standard_normal(n)
    wtw, wty, yty = oracle.precompute(grid, X, y)
    W = dense_w_textbook(grid, X)
    A = oracle.wtw_dense_from_dia(grid, wtw)
    np.testing.assert_allclose(A, W.T @ W, atol=1e-12 * n)
    np.testing.assert_allclose(wty, W.T @ y, atol=1e-12 * n)
    assert abs(yty - y @ y) <= 1e-12 * n
    # the DIA layout holds every nonzero: at most 7^d per row (Claim 2)
    assert np.count_nonzero(np.abs(W.T @ W) > 1e-14, axis=1).max() <= 7 ** len(m)


@pytest.mark.parametrize("m", [[11], [7, 9], [6, 5, 7]])
def test_linear_wtw_bruteforce_dense(m):
    """Linear interpolation (Sec. 2.3: 2^d nonzeros per row of W): the
    statistics equal the brute-force hat-function W, and W^T W has at most
    3^d nonzeros per row, all within offsets -1..1 (Claim 2, r = 1)."""
    rng = np.random.default_rng(10 + len(m))
    grid = oracle.make_grid(m, origin=[0.5] * len(m), spacing=[0.3] * len(m))
    grid["interp"] = "linear"
    n = 400
    X = rand_points(rng, grid, n)
    y = rng.standard_normal(n)
    wtw, wty, yty = oracle.precompute(grid, X, y)
    W = dense_w_textbook(grid, X)
    assert np.count_nonzero(W, axis=1).max() <= 2 ** len(m)
    A = oracle.wtw_dense_from_dia(grid, wtw)
    np.testing.assert_allclose(A, W.T @ W, atol=1e-12 * n)
    np.testing.assert_allclose(wty, W.T @ y, atol=1e-12 * n)
    np.testing.assert_allclose(oracle.dense_w(grid, X), W, atol=1e-14)
    d = len(m)
    offs = np.array(np.unravel_index(np.arange(7 ** d), (7,) * d)).T - 3
    outer = np.abs(offs).max(axis=1) > 1
    assert np.all(wtw[:, outer] == 0.0)
    assert np.count_nonzero(np.abs(W.T @ W) > 1e-14, axis=1).max() <= 3 ** d


def test_linear_reproduces_affine_only():
    """Linear interpolation is exact for affine functions and not for a
    quadratic (which the cubic Keys weights do reproduce)."""
    rng = np.random.default_rng(4)
    grid = oracle.make_grid([9, 8], origin=[0.0, 1.0], spacing=[0.5, 0.25])
    X = rand_points(rng, grid, 200)
    coords = np.array(np.unravel_index(np.arange(72), (9, 8)), float)
    G = np.array([grid["origin"][k] + coords[k] * grid["spacing"][k] for k in range(2)])
    aff = 0.7 - 1.3 * G[0] + 2.1 * G[1]
    quad = G[0] ** 2
    lin = dict(grid, interp="linear")
    Wl = oracle.dense_w(lin, X)
    Wc = oracle.dense_w(grid, X)
    np.testing.assert_allclose(Wl @ aff, 0.7 - 1.3 * X[0] + 2.1 * X[1], atol=1e-12)
    np.testing.assert_allclose(Wc @ quad, X[0] ** 2, atol=1e-12)
    assert np.abs(Wl @ quad - X[0] ** 2).max() > 1e-3


def test_wtw_invariants():
    rng = np.random.default_rng(5)
    grid = oracle.make_grid([8, 10], origin=[0.0, 0.0], spacing=[1.0, 0.5])
    n = 2000
    X = rand_points(rng, grid, n)
    y = rng.standard_normal(n)
    wtw, wty, yty = oracle.precompute(grid, X, y)
    A = oracle.wtw_dense_from_dia(grid, wtw)
    M = A.shape[0]
    np.testing.assert_allclose(A, A.T, atol=1e-12)
    assert np.linalg.eigvalsh(A).min() >= -1e-12 * np.abs(A).max()
    ones = np.ones(M)
    _, w1, _ = oracle.precompute(grid, X, np.ones(n))
    np.testing.assert_allclose(A @ ones, w1, atol=1e-10)
    assert abs(ones @ A @ ones - n) < 1e-8
    assert abs(wty.sum() - y.sum()) < 1e-9
    _, wts, _ = oracle.stencils(grid, X)
    assert abs(np.trace(A) - (wts ** 2).sum()) < 1e-9
    np.testing.assert_allclose(oracle.wtw_matvec(grid, wtw, ones), A @ ones, atol=1e-12)


def test_points_on_nodes_give_diagonal_histogram():
    grid = oracle.make_grid([9, 6], origin=[0.0, 0.0], spacing=[1.0, 1.0])
    rng = np.random.default_rng(1)
    i0 = rng.integers(1, 8, 500)
    i1 = rng.integers(1, 5, 500)
    X = np.array([i0, i1], float)
    wtw, wty, _ = oracle.precompute(grid, X, np.ones(500))
    A = oracle.wtw_dense_from_dia(grid, wtw)
    hist = np.zeros((9, 6))
    np.add.at(hist, (i0, i1), 1.0)
    np.testing.assert_allclose(A, np.diag(hist.ravel()), atol=1e-13)


def test_probe_generator_published_vectors():
    rows = [l.split() for l in open(os.path.join(GOLD, "splitmix64_seed0.txt"))
            if not l.startswith("#")]
    for c, out in rows:
        assert oracle.splitmix64(int(c, 16)) == int(out, 16)
    z = oracle.probe_values(4, 3, 1000)
    assert set(np.unique(z)) == {-1.0, 1.0}
    assert abs(z.mean()) < 0.15


def test_probe_sketches_match_dense():
    rng = np.random.default_rng(2)
    grid = oracle.make_grid([7, 8], origin=[0.0, 0.0], spacing=[1.0, 1.0])
    X = rand_points(rng, grid, 300)
    S = oracle.probe_sketches(grid, X, 7, 3)
    W = dense_w_textbook(grid, X)
    for j in range(3):
        z = oracle.probe_values(7, j, 300)
        np.testing.assert_allclose(S[j], W.T @ z, atol=1e-11)


# --------------------------------------------------------------------------
# K_G (Sec. 2.3: multilevel Toeplitz for a stationary kernel on a grid).
# --------------------------------------------------------------------------
def test_kg_matvec_vs_kernel_on_grid_points():
    grid = oracle.make_grid([9, 6, 5], origin=[0.1, -0.2, 0.0], spacing=[0.07, 0.11, 0.05])
    hyp = {"lengthscale": [0.13, 0.2, 0.09], "outputscale": 1.7, "noise": 0.1}
    coords = np.array(np.meshgrid(*[grid["origin"][k] + grid["spacing"][k] * np.arange(grid["m"][k])
                                    for k in range(3)], indexing="ij")).reshape(3, -1).T
    K = oracle.se_kernel(coords, coords, hyp["lengthscale"], hyp["outputscale"])
    np.testing.assert_allclose(oracle.kg_dense(grid, hyp), K, atol=1e-13)
    v = np.random.default_rng(0).standard_normal(K.shape[0])
    np.testing.assert_allclose(oracle.kg_matvec(grid, hyp, v), K @ v, atol=1e-12)


def test_dkg_matvec_vs_finite_difference():
    grid = oracle.make_grid([8, 7], origin=[0.0, 0.0], spacing=[0.1, 0.1])
    hyp = {"lengthscale": [0.2, 0.3], "outputscale": 1.3, "noise": 0.1}
    v = np.random.default_rng(1).standard_normal(56)
    for which in range(3):
        h = 1e-6
        hp = {k: (list(v_) if isinstance(v_, list) else v_) for k, v_ in hyp.items()}
        hm = {k: (list(v_) if isinstance(v_, list) else v_) for k, v_ in hyp.items()}
        if which < 2:
            hp["lengthscale"][which] *= np.exp(h)
            hm["lengthscale"][which] *= np.exp(-h)
        else:
            hp["outputscale"] *= np.exp(h)
            hm["outputscale"] *= np.exp(-h)
        fd = (oracle.kg_matvec(grid, hp, v) - oracle.kg_matvec(grid, hm, v)) / (2 * h)
        np.testing.assert_allclose(oracle.dkg_matvec(grid, hyp, v, which), fd, rtol=1e-6, atol=1e-8)


# --------------------------------------------------------------------------
# Solves: Theorem 1 / Claim 5 (m-space mean == SKI mean), Prop. 1.
# --------------------------------------------------------------------------
def small_problem(seed=0, m=(14, 12), n=600):
    rng = np.random.default_rng(seed)
    grid = oracle.make_grid(list(m), lo=0.0, hi=1.0)
    X = rng.uniform(0, 1, (len(m), n))
    y = np.sin(4 * X[0]) + (np.cos(3 * X[1]) if len(m) > 1 else 0) + 0.1 * rng.standard_normal(n)
    hyp = {"lengthscale": [0.2] * len(m), "outputscale": 1.2, "noise": 0.3}
    return grid, X, y, hyp


@pytest.mark.parametrize("interp", ["cubic", "linear"])
@pytest.mark.parametrize("m", [(30,), (14, 12), (6, 7, 5)])
def test_m_space_mean_equals_dense_ski(m, interp):
    grid, X, y, hyp = small_problem(1, m, 500)
    grid["interp"] = interp
    wtw, wty, yty = oracle.precompute(grid, X, y)
    mu, wtz, info = oracle.solve_mean(grid, hyp, wtw, wty, yty, tol=1e-13)
    mu_d, z_d, W = oracle.ski_dense_mean(grid, hyp, X, y)
    np.testing.assert_allclose(mu, mu_d, rtol=0, atol=1e-10 * np.abs(mu_d).max())
    np.testing.assert_allclose(wtz, W.T @ z_d, atol=1e-9 * np.abs(W.T @ z_d).max())
    xq = np.random.default_rng(9).uniform(0.1, 0.9, (len(m), 50))
    np.testing.assert_allclose(oracle.interpolate(grid, mu, xq),
                               oracle.dense_w(grid, xq) @ mu_d, atol=1e-9)


def test_factorized_cg_iterates_equal_plain_cg():
    """Prop. 1: Alg. 1 on the n x n SKI system, from x_0 = y / sigma^2, has
    the same iterates as the factorized algorithm (compared through W^T x_k)."""
    grid, X, y, hyp = small_problem(2, (10, 9), 300)
    wtw, wty, yty = oracle.precompute(grid, X, y)
    _, _, info = oracle.solve_mean(grid, hyp, wtw, wty, yty, tol=1e-10, history=True)
    W = oracle.dense_w(grid, X)
    A = W @ oracle.kg_dense(grid, hyp) @ W.T + hyp["noise"] ** 2 * np.eye(300)
    x = y / hyp["noise"] ** 2
    r = y - A @ x
    p = r.copy()
    hist = [W.T @ x]
    rr = r @ r
    for k in range(1000):
        Ap = A @ p
        a = rr / (p @ Ap)
        x = x + a * p
        r = r - a * Ap
        hist.append(W.T @ x)
        rn = r @ r
        if rn <= 1e-20 * (y @ y):
            break
        p = r + (rn / rr) * p
        rr = rn
    # exact agreement while rounding has not yet been amplified by the loss of
    # orthogonality of finite-precision CG
    for k in range(8):
        np.testing.assert_allclose(info["wtx_history"][k], hist[k],
                                   atol=1e-10 * np.abs(hist[-1]).max())
    # both reach the same solution; iteration counts differ only through
    # rounding (the paper reports near-identical counts)
    np.testing.assert_allclose(info["wtx_history"][-1], hist[-1],
                               atol=1e-6 * np.abs(hist[-1]).max())
    n_plain = len(hist) - 1
    assert info["iterations"] <= 1.5 * n_plain + 2


def test_grid_rhs_solve():
    grid, X, y, hyp = small_problem(3, (9, 8), 250)
    wtw, _, _ = oracle.precompute(grid, X, y)
    yhat = np.random.default_rng(0).standard_normal(72)
    xd, _ = oracle.solve_grid_rhs(grid, hyp, wtw, yhat, tol=1e-13)
    W = oracle.dense_w(grid, X)
    A = W @ oracle.kg_dense(grid, hyp) @ W.T + hyp["noise"] ** 2 * np.eye(250)
    ref = W.T @ np.linalg.solve(A, W @ yhat)
    np.testing.assert_allclose(xd, ref, atol=1e-9 * np.abs(ref).max())


def test_ski_mean_converges_to_exact_gp():
    """(iii) The SKI mean approaches the exact GP mean (Fact 1) as the grid is
    refined; Keys' kernel is third order, so halving h cuts the error >= 4x
    until it levels off."""
    rng = np.random.default_rng(0)
    n = 400
    x = rng.uniform(0, 1, n)
    y = np.sin(6 * np.pi * x) + 0.5 * np.sin(20 * np.pi * x) + 0.1 * rng.standard_normal(n)
    ell, s, sig = 0.05, 1.0, 0.1
    xq = np.linspace(0.05, 0.95, 200)
    exact = oracle.exact_gp_mean(x[:, None], y, xq[:, None], [ell], s, sig)
    errs = []
    for m in (40, 80, 160):
        grid = oracle.make_grid([m], lo=0.0, hi=1.0)
        wtw, wty, yty = oracle.precompute(grid, x, y)
        mu, _, _ = oracle.solve_mean(grid, {"lengthscale": [ell], "outputscale": s, "noise": sig},
                                     wtw, wty, yty, tol=1e-12)
        errs.append(np.abs(oracle.interpolate(grid, mu, xq) - exact).max())
    assert errs[1] < errs[0] / 4 and errs[2] < errs[1] / 4, errs


# --------------------------------------------------------------------------
# Log likelihood: Claim 6, Fact 2 == Def. 2, gradient, SLQ.
# --------------------------------------------------------------------------
def test_claim6_logdet_shift_and_fact2_equals_def2():
    grid, X, y, hyp = small_problem(4, (8, 7), 200)
    wtw, wty, yty = oracle.precompute(grid, X, y)
    W = oracle.dense_w(grid, X)
    KG = oracle.kg_dense(grid, hyp)
    s2 = hyp["noise"] ** 2
    n, M = W.shape
    ld_n = np.linalg.slogdet(W @ KG @ W.T + s2 * np.eye(n))[1]
    ld_m = np.linalg.slogdet(KG @ (W.T @ W) + s2 * np.eye(M))[1]
    assert abs(ld_n - (ld_m + (n - M) * np.log(s2))) < 1e-8 * abs(ld_n)
    a = oracle.gsgp_mll_fact2(grid, hyp, wtw, wty, yty, n)
    b = oracle.ski_dense_mll(grid, hyp, X, y)
    assert abs(a - b) < 1e-8 * abs(b)


def _fd_grad(f, hyp, d, h=1e-5):
    g = np.zeros(d + 2)
    for th in range(d + 2):
        def shifted(e):
            hp = {"lengthscale": list(hyp["lengthscale"]), "outputscale": hyp["outputscale"],
                  "noise": hyp["noise"], "kernel": hyp.get("kernel", "se")}
            if th < d:
                hp["lengthscale"][th] *= np.exp(e)
            elif th == d:
                hp["outputscale"] *= np.exp(e)
            else:
                hp["noise"] *= np.exp(e)
            return f(hp)
        g[th] = (shifted(h) - shifted(-h)) / (2 * h)
    return g


def test_dense_gradient_vs_finite_differences():
    grid, X, y, hyp = small_problem(5, (7, 6), 120)
    g = oracle.ski_dense_grad(grid, hyp, X, y)
    fd = _fd_grad(lambda hp: oracle.ski_dense_mll(grid, hp, X, y), hyp, 2)
    np.testing.assert_allclose(g, fd, rtol=1e-5, atol=1e-6)


def test_mll_exact_trace_gradient_and_quadratic_term():
    grid, X, y, hyp = small_problem(6, (7, 6), 150)
    wtw, wty, yty = oracle.precompute(grid, X, y)
    sk = oracle.probe_sketches(grid, X, 11, 4)
    mll, g, info = oracle.mll_and_grad(grid, hyp, wtw, wty, yty, 150, sk,
                                       exact_trace=True, tol=1e-13)
    np.testing.assert_allclose(g, oracle.ski_dense_grad(grid, hyp, X, y), rtol=1e-7, atol=1e-8)
    W = oracle.dense_w(grid, X)
    A = W @ oracle.kg_dense(grid, hyp) @ W.T + hyp["noise"] ** 2 * np.eye(150)
    assert abs(info["q"] - y @ np.linalg.solve(A, y)) < 1e-8 * abs(info["q"])


def test_lanczos_from_cg_matches_dense_lanczos():
    grid, X, y, hyp = small_problem(7, (6, 7), 160)
    wtw, _, _ = oracle.precompute(grid, X, y)
    z = oracle.probe_values(3, 0, 160)
    bhat = oracle.probe_sketches(grid, X, 3, 1)[0]
    _, info = oracle.fcg_probe(grid, hyp, wtw, bhat, 160.0, tol=1e-14, maxiter=12)
    T_cg = oracle.lanczos_from_cg(info["alpha"], info["beta"], 10)
    W = oracle.dense_w(grid, X)
    A = W @ oracle.kg_dense(grid, hyp) @ W.T + hyp["noise"] ** 2 * np.eye(160)
    T_l, _ = oracle.lanczos_dense(A, z, 10)
    np.testing.assert_allclose(T_cg, T_l, atol=1e-8 * np.abs(T_l).max())


def test_fcg_probe_iterates_equal_dense_cg():
    grid, X, y, hyp = small_problem(8, (7, 7), 180)
    wtw, _, _ = oracle.precompute(grid, X, y)
    z = oracle.probe_values(5, 1, 180)
    bhat = oracle.probe_sketches(grid, X, 5, 2)[1]
    wx, info = oracle.fcg_probe(grid, hyp, wtw, bhat, 180.0, tol=1e-12, history=True)
    W = oracle.dense_w(grid, X)
    A = W @ oracle.kg_dense(grid, hyp) @ W.T + hyp["noise"] ** 2 * np.eye(180)
    x = np.zeros(180); r = z.copy(); p = r.copy(); rr = r @ r
    for k in range(10):
        Ap = A @ p
        a = rr / (p @ Ap)
        x += a * p; r -= a * Ap
        np.testing.assert_allclose(info["wtx_history"][k], W.T @ x, atol=1e-9 * np.abs(W.T @ x).max())
        rn = r @ r; p = r + rn / rr * p; rr = rn
    np.testing.assert_allclose(wx, W.T @ np.linalg.solve(A, z), atol=1e-8 * np.abs(wx).max())


def test_slq_logdet_unbiased():
    grid, X, y, hyp = small_problem(9, (6, 6), 120)
    wtw, wty, yty = oracle.precompute(grid, X, y)
    W = oracle.dense_w(grid, X)
    A = W @ oracle.kg_dense(grid, hyp) @ W.T + hyp["noise"] ** 2 * np.eye(120)
    exact = np.linalg.slogdet(A)[1]
    sk = oracle.probe_sketches(grid, X, 21, 200)
    _, _, info = oracle.mll_and_grad(grid, hyp, wtw, wty, yty, 120, sk, lanczos_steps=30)
    samples = info["logdet_samples"]
    se = samples.std(ddof=1) / np.sqrt(len(samples))
    assert abs(samples.mean() - exact) < 4 * se + 1e-6 * abs(exact), (samples.mean(), exact, se)


def test_mll_value_with_unit_probes_equals_dense_def2():
    """Pins the assembled value -1/2 (logdet + q + n log 2 pi) deterministically
    (Fact 2 / Def. 2).  With the n probes z_i = sqrt(n) e_i (||z_i||^2 = n,
    as for a Rademacher probe) and each probe's Lanczos run until its Krylov
    space is exhausted (A = W K_G W^T + s2 I is a rank-M update of s2 I, so
    at most M + 1 steps), Gauss quadrature gives e_i^T log(A) e_i exactly and
    the estimator sums to tr log A = logdet A: the oracle's MLL must then
    equal the Cholesky MLL of Def. 2.  A dropped n log 2 pi, a sign slip or
    a wrong factor on q or on the log-determinant fails this test."""
    for seed, m, n in ((12, (6, 5), 90), (13, (20,), 70)):
        grid, X, y, hyp = small_problem(seed, m, n)
        wtw, wty, yty = oracle.precompute(grid, X, y)
        sk = np.sqrt(n) * oracle.dense_w(grid, X)      # rows: W^T (sqrt(n) e_i)
        mll, _, info = oracle.mll_and_grad(grid, hyp, wtw, wty, yty, n, sk,
                                           lanczos_steps=10 ** 6, tol=1e-13, maxiter=400)
        W = oracle.dense_w(grid, X)
        A = W @ oracle.kg_dense(grid, hyp) @ W.T + hyp["noise"] ** 2 * np.eye(n)
        exact_logdet = np.linalg.slogdet(A)[1]
        ref = oracle.ski_dense_mll(grid, hyp, X, y)
        assert abs(info["logdet"] - exact_logdet) <= 1e-9 * abs(exact_logdet), (
            info["logdet"], exact_logdet)
        assert abs(mll - ref) <= 1e-9 * abs(ref), (mll, ref)


def test_mll_value_rademacher_within_standard_errors():
    """The same value with 256 Rademacher probes and full-length Lanczos:
    unbiased (Hutchinson), so it lands within 4 standard errors (from the
    per-probe log-determinant samples) of the Def. 2 MLL."""
    grid, X, y, hyp = small_problem(14, (7, 6), 130)
    wtw, wty, yty = oracle.precompute(grid, X, y)
    sk = oracle.probe_sketches(grid, X, 41, 256)
    mll, _, info = oracle.mll_and_grad(grid, hyp, wtw, wty, yty, 130, sk,
                                       lanczos_steps=10 ** 6, tol=1e-12, maxiter=400)
    ref = oracle.ski_dense_mll(grid, hyp, X, y)
    se = 0.5 * info["logdet_samples"].std(ddof=1) / np.sqrt(256)
    assert abs(mll - ref) <= 4 * se + 1e-9 * abs(ref), (mll, ref, se)


def test_hutchinson_gradient_close_to_exact():
    grid, X, y, hyp = small_problem(10, (6, 6), 140)
    wtw, wty, yty = oracle.precompute(grid, X, y)
    sk = oracle.probe_sketches(grid, X, 31, 64)
    _, g_h, _ = oracle.mll_and_grad(grid, hyp, wtw, wty, yty, 140, sk)
    g_e = oracle.ski_dense_grad(grid, hyp, X, y)
    # loose statistical agreement (64 probes)
    assert np.all(np.abs(g_h - g_e) < 0.25 * np.abs(g_e) + 2.0), (g_h, g_e)


# --------------------------------------------------------------------------
# Other product stationary kernels (Matern 1/2, 3/2, 5/2; Sec. 2.3).
# --------------------------------------------------------------------------
MATERN_NU = {"matern12": 0.5, "matern32": 1.5, "matern52": 2.5}


@pytest.mark.parametrize("kind", sorted(MATERN_NU))
def test_matern_closed_forms_match_bessel_definition(kind):
    """The Matern kernel of smoothness nu, 2^(1-nu)/Gamma(nu) (sqrt(2 nu) r)^nu
    K_nu(sqrt(2 nu) r) through scipy's modified Bessel function, equals the
    oracle's closed form (and 1 at r = 0)."""
    from scipy.special import gamma, kv
    nu = MATERN_NU[kind]
    r = np.linspace(1e-3, 6.0, 400)
    z = np.sqrt(2 * nu) * r
    ref = 2 ** (1 - nu) / gamma(nu) * z ** nu * kv(nu, z)
    np.testing.assert_allclose(oracle.kernel_1d(r, kind), ref, rtol=1e-12, atol=1e-15)
    assert oracle.kernel_1d(0.0, kind) == 1.0


@pytest.mark.parametrize("kind", ["se"] + sorted(MATERN_NU))
def test_kernel_log_lengthscale_derivative(kind):
    """d/dlog l of k1(|x|/l) by central differences in log l."""
    x = np.linspace(0.0, 2.0, 101)
    ell, h = 0.37, 1e-6
    fd = (oracle.kernel_1d(x / (ell * np.exp(h)), kind)
          - oracle.kernel_1d(x / (ell * np.exp(-h)), kind)) / (2 * h)
    np.testing.assert_allclose(oracle.kernel_1d_dlog_ell(x / ell, kind), fd, rtol=1e-6,
                               atol=1e-10)


def test_matern12_grid_precision_is_tridiagonal():
    """On an equispaced grid the Matern-1/2 (exponential) kernel matrix is
    rho^|i-j| with rho = exp(-h/l), whose inverse is the tridiagonal AR(1)
    precision (1/(1-rho^2)) tridiag(-rho, (1, 1+rho^2, ..., 1+rho^2, 1), -rho)."""
    m, h, ell = 25, 0.05, 0.3
    grid = oracle.make_grid([m], origin=[0.0], spacing=[h])
    hyp = {"lengthscale": [ell], "outputscale": 1.0, "noise": 0.1, "kernel": "matern12"}
    K = oracle.kg_dense(grid, hyp)
    rho = np.exp(-h / ell)
    Q = np.diag(np.r_[1.0, np.full(m - 2, 1 + rho * rho), 1.0])
    Q += np.diag(np.full(m - 1, -rho), 1) + np.diag(np.full(m - 1, -rho), -1)
    Q /= 1 - rho * rho
    np.testing.assert_allclose(K @ Q, np.eye(m), atol=1e-12)


@pytest.mark.parametrize("kind", sorted(MATERN_NU))
def test_matern_kg_matvec_and_gradient(kind):
    """K_G by circulant embedding equals the dense product-kernel matrix on
    the grid points, and the dense SKI gradient matches finite differences of
    the dense log likelihood for the Matern kernels."""
    grid = oracle.make_grid([9, 7], origin=[0.1, -0.2], spacing=[0.07, 0.11])
    hyp = {"lengthscale": [0.13, 0.2], "outputscale": 1.7, "noise": 0.1, "kernel": kind}
    coords = np.array(np.meshgrid(*[grid["origin"][k] + grid["spacing"][k] * np.arange(grid["m"][k])
                                    for k in range(2)], indexing="ij")).reshape(2, -1).T
    K = hyp["outputscale"] * np.prod(
        [oracle.kernel_1d(np.abs(coords[:, None, k] - coords[None, :, k]) / hyp["lengthscale"][k],
                          kind) for k in range(2)], axis=0)
    np.testing.assert_allclose(oracle.kg_dense(grid, hyp), K, atol=1e-13)
    v = np.random.default_rng(2).standard_normal(K.shape[0])
    np.testing.assert_allclose(oracle.kg_matvec(grid, hyp, v), K @ v, atol=1e-12)
    g2, X, y, h2 = small_problem(7, (7, 6), 120)
    h2["kernel"] = kind
    g = oracle.ski_dense_grad(g2, h2, X, y)
    fd = _fd_grad(lambda hp: oracle.ski_dense_mll(g2, hp, X, y), h2, 2)
    np.testing.assert_allclose(g, fd, rtol=1e-5, atol=1e-6)


def test_ski_posterior_covariance_information_form():
    """SKI as Bayesian linear regression on the grid values (f_G ~ N(0, K_G),
    y = W f_G + noise): the posterior covariance of f_G is
    (K_G^{-1} + W^T W / sigma^2)^{-1}, so the covariance between query points
    is Wq (K_G^{-1} + W^T W / sigma^2)^{-1} Wq^T; the oracle's covariance form
    (Woodbury) must agree, and the matrix is symmetric positive definite."""
    grid, X, y, hyp = small_problem(8, (9, 8), 200)
    rng = np.random.default_rng(9)
    Xq = rand_points(rng, grid, 12)
    C = oracle.ski_dense_cov(grid, hyp, X, Xq)
    W = oracle.dense_w(grid, X)
    Wq = oracle.dense_w(grid, Xq)
    KG = oracle.kg_dense(grid, hyp)
    S = np.linalg.inv(np.linalg.inv(KG) + W.T @ W / hyp["noise"] ** 2)
    np.testing.assert_allclose(C, Wq @ S @ Wq.T, rtol=1e-7, atol=1e-10)
    np.testing.assert_allclose(C, C.T, atol=1e-12)
    assert np.linalg.eigvalsh(C).min() > 0


# --------------------------------------------------------------------------
# Factorized Lanczos (Algs. 6-7) and the rank-k covariance built on it.
# --------------------------------------------------------------------------
def test_efla_matches_dense_lanczos():
    """The factorized iterates Q_i = W qh_i + d_i y reproduce plain Lanczos
    with one reorthogonalisation pass on the dense A = W K_G W^T + s2 I."""
    grid, X, y, hyp = small_problem(8, (9, 8), 200)
    wtw, wty, yty = oracle.precompute(grid, X, y)
    W = oracle.dense_w(grid, X)
    A = W @ oracle.kg_dense(grid, hyp) @ W.T + hyp["noise"] ** 2 * np.eye(W.shape[0])
    T_d, Q_d = oracle.lanczos_dense(A, y, 15)
    al, be, Qh, P, d = oracle.efla(grid, hyp, wtw, wty, yty, 15, reorth=1)
    T = np.diag(al) + np.diag(be, 1) + np.diag(be, -1)
    np.testing.assert_allclose(T, T_d, rtol=1e-9, atol=1e-9 * np.abs(T_d).max())
    Q = W @ Qh.T + np.outer(y, d)
    np.testing.assert_allclose(Q, Q_d, atol=1e-9)
    np.testing.assert_allclose(P, Qh @ (W.T @ W), atol=1e-10)


def test_efla_orthonormal_and_projects_A():
    """With two passes the Lanczos vectors stay orthonormal in n-space over
    many steps, and Q^T A Q is the tridiagonal T."""
    grid, X, y, hyp = small_problem(3, (11, 10), 300)
    wtw, wty, yty = oracle.precompute(grid, X, y)
    W = oracle.dense_w(grid, X)
    A = W @ oracle.kg_dense(grid, hyp) @ W.T + hyp["noise"] ** 2 * np.eye(W.shape[0])
    al, be, Qh, P, d = oracle.efla(grid, hyp, wtw, wty, yty, 60)
    Q = W @ Qh.T + np.outer(y, d)
    k = Q.shape[1]
    np.testing.assert_allclose(Q.T @ Q, np.eye(k), atol=1e-9)
    T = np.diag(al) + np.diag(be, 1) + np.diag(be, -1)
    np.testing.assert_allclose(Q.T @ A @ Q, T, atol=1e-8 * np.abs(T).max())


def test_love_cov_full_rank_is_exact():
    """Once the Krylov space is exhausted it holds range(W), so the rank-k
    covariance equals the exact SKI covariance (Def. 2)."""
    grid, X, y, hyp = small_problem(8, (9, 8), 200)
    wtw, wty, yty = oracle.precompute(grid, X, y)
    Xq = rand_points(np.random.default_rng(2), grid, 10)
    M = oracle.grid_size(grid)
    al, _, _, _, _ = oracle.efla(grid, hyp, wtw, wty, yty, M + 1)
    assert len(al) <= M + 1
    C = oracle.love_cov(grid, hyp, wtw, wty, yty, Xq, M + 1)
    ref = oracle.ski_dense_cov(grid, hyp, X, Xq)
    np.testing.assert_allclose(C, ref, rtol=0, atol=1e-8 * np.abs(np.diag(ref)).max())


def test_love_variance_decreases_with_rank():
    """u^T T^{-1} u is the A^{-1}-norm of the projection of W K_G w_x onto a
    growing Krylov space: the rank-k variances fall with k and stay above
    the exact ones."""
    grid, X, y, hyp = small_problem(5, (12, 10), 400)
    wtw, wty, yty = oracle.precompute(grid, X, y)
    Xq = rand_points(np.random.default_rng(4), grid, 15)
    exact = np.diag(oracle.ski_dense_cov(grid, hyp, X, Xq))
    prev = None
    for k in (3, 8, 20, 50):
        v = np.diag(oracle.love_cov(grid, hyp, wtw, wty, yty, Xq, k))
        assert np.all(v >= exact - 1e-10)
        if prev is not None:
            assert np.all(v <= prev + 1e-10)
        prev = v


# --------------------------------------------------------------------------
# The OpenMP timing variants of the oracle (all-cores CPU baseline).
# --------------------------------------------------------------------------
@pytest.mark.parametrize("m", [(50,), (20, 17), (9, 8, 7)])
def test_openmp_oracle_equals_serial(m):
    """Per-thread chunks combined in thread order: the statistics equal the
    serial ones to rounding and repeat bit for bit; the banded product splits
    rows only, so it equals the serial product exactly; an out-of-grid point
    is reported with its global index."""
    d = len(m)
    grid = oracle.make_grid(list(m), lo=0.0, hi=1.0)
    rng = np.random.default_rng(17)
    X = rng.uniform(0, 1, (d, 20011))
    y = rng.standard_normal(20011)
    a = oracle.precompute(grid, X, y)
    b = oracle.precompute(grid, X, y, threads=5)
    c = oracle.precompute(grid, X, y, threads=5)
    assert np.abs(a[0] - b[0]).max() <= 1e-13 * np.abs(a[0]).max()
    assert np.abs(a[1] - b[1]).max() <= 1e-13 * np.abs(a[1]).max()
    assert abs(a[2] - b[2]) <= 1e-13 * a[2]
    assert np.array_equal(b[0], c[0]) and np.array_equal(b[1], c[1]) and b[2] == c[2]
    v = rng.standard_normal(a[1].shape[0])
    assert np.array_equal(oracle.wtw_matvec(grid, a[0], v), oracle.wtw_matvec(grid, a[0], v, threads=4))
    X[d - 1, 15000] = 5.0
    with pytest.raises(oracle.native.OutOfGrid, match="15000"):
        oracle.precompute(grid, X, y, threads=3)


def test_oracle_c_under_address_and_ub_sanitizers(tmp_path):
    """The oracle's C code built with -fsanitize=address,undefined and run
    through every entry point (serial and threaded, both interpolation
    schemes, 1-3 dimensions, error paths): no invalid access, leak or
    undefined behaviour, and the invariants hold."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    here = os.path.join(os.path.dirname(os.path.dirname(__file__)), "oracle")
    exe = str(tmp_path / "oracle_sanitize_check")
    cmd = ["gcc", "-O1", "-g", "-std=c99", "-fopenmp", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-ffp-contract=off",
           os.path.join(here, "precompute.c"), os.path.join(here, "sanitize_check.c"),
           "-lm", "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all checks passed" in r.stdout


# --------------------------------------------------------------------------
# Reverse-mode derivative of the stochastic Lanczos log-determinant (the
# gradient of the estimate itself, through each probe's Lanczos steps).
# --------------------------------------------------------------------------
def _hyp_shift(hyp, i, d, e):
    hp = {"lengthscale": list(hyp["lengthscale"]), "outputscale": hyp["outputscale"],
          "noise": hyp["noise"]}
    f = np.exp(e)
    if i < d:
        hp["lengthscale"][i] *= f
    elif i == d:
        hp["outputscale"] *= f
    else:
        hp["noise"] *= f
    return hp


def test_logm_e1_gradient_vs_finite_differences():
    rng = np.random.default_rng(3)
    k = 9
    al = 2.0 + rng.uniform(0, 1, k)
    be = 0.5 * rng.uniform(0.1, 1, k - 1)
    T = np.diag(al) + np.diag(be, 1) + np.diag(be, -1)
    ga, gb = oracle.logm_e1_grad(T)
    h = 1e-6
    for i in range(k):
        E = np.zeros((k, k)); E[i, i] = h
        fd = (oracle.logm_e1(T + E) - oracle.logm_e1(T - E)) / (2 * h)
        assert abs(ga[i] - fd) <= 1e-8
    for i in range(k - 1):
        E = np.zeros((k, k)); E[i, i + 1] = E[i + 1, i] = h
        fd = (oracle.logm_e1(T + E) - oracle.logm_e1(T - E)) / (2 * h)
        assert abs(gb[i] - fd) <= 1e-8


def _dense_A(grid, X, hp):
    W = oracle.dense_w(grid, X)
    return W @ oracle.kg_dense(grid, hp) @ W.T + hp["noise"] ** 2 * np.eye(X.shape[1])


@pytest.mark.parametrize("k", [10, 30])
def test_slq_gradient_dense_vs_finite_differences(k):
    """The reverse sweep through k plain Lanczos steps equals central
    differences (h = 1e-4) of the same deterministic k-step value."""
    grid, X, y, hyp = small_problem(21, (7, 6), 150)
    n = X.shape[1]
    z = oracle.probe_values(3, 0, n)
    A = _dense_A(grid, X, hyp)
    eps = 1e-6
    dA = [(_dense_A(grid, X, _hyp_shift(hyp, i, 2, eps)) - _dense_A(grid, X, _hyp_shift(hyp, i, 2, -eps)))
          / (2 * eps) for i in range(4)]
    val, g = oracle.slq_logdet_grad_dense(A, dA, z, k)
    h = 1e-4
    for i in range(4):
        fp, _ = oracle.slq_logdet_grad_dense(_dense_A(grid, X, _hyp_shift(hyp, i, 2, h)), [], z, k)
        fm, _ = oracle.slq_logdet_grad_dense(_dense_A(grid, X, _hyp_shift(hyp, i, 2, -h)), [], z, k)
        fd = (fp - fm) / (2 * h)
        assert abs(g[i] - fd) <= 1e-6 * np.abs(g).max(), (i, g[i], fd)


def test_slq_gradient_factorized_equals_dense():
    """The m-space form (CG coefficients, Lanczos vectors from the factorized
    CG residuals, compressed inner products) equals the dense n-space sweep:
    value and gradient."""
    for seed, m, n, k in ((22, (7, 6), 160, 10), (23, (25,), 120, 12)):
        grid, X, y, hyp = small_problem(seed, m, n)
        d = grid["d"]
        wtw, _, _ = oracle.precompute(grid, X, y)
        z = oracle.probe_values(5, 1, n)
        bhat = oracle.probe_sketches(grid, X, 5, 2)[1]
        A = _dense_A(grid, X, hyp)
        eps = 1e-6
        dA = [(_dense_A(grid, X, _hyp_shift(hyp, i, d, eps))
               - _dense_A(grid, X, _hyp_shift(hyp, i, d, -eps))) / (2 * eps) for i in range(d + 2)]
        v_d, g_d = oracle.slq_logdet_grad_dense(A, dA, z, k)
        v_f, g_f = oracle.slq_logdet_grad(grid, hyp, wtw, bhat, n, k)
        assert abs(v_f - v_d) <= 1e-10 * abs(v_d)
        np.testing.assert_allclose(g_f, g_d, rtol=0, atol=1e-7 * np.abs(g_d).max())


def test_mll_slq_gradient_matches_finite_differences_of_its_value():
    """With slq_grad the oracle's gradient is that of its own (stochastic)
    MLL value: central differences of mll_and_grad's MLL with the same
    probes agree tightly, where the Hutchinson gradient differs by the
    estimator's noise."""
    grid, X, y, hyp = small_problem(24, (8, 7), 300)
    n = X.shape[1]
    wtw, wty, yty = oracle.precompute(grid, X, y)
    sk = oracle.probe_sketches(grid, X, 9, 4)
    kw = dict(lanczos_steps=15, tol=1e-12, maxiter=2000)
    _, g, _ = oracle.mll_and_grad(grid, hyp, wtw, wty, yty, n, sk, slq_grad=True, **kw)
    h = 1e-4
    for i in range(4):
        fp, _, _ = oracle.mll_and_grad(grid, _hyp_shift(hyp, i, 2, h), wtw, wty, yty, n, sk, **kw)
        fm, _, _ = oracle.mll_and_grad(grid, _hyp_shift(hyp, i, 2, -h), wtw, wty, yty, n, sk, **kw)
        fd = (fp - fm) / (2 * h)
        assert abs(g[i] - fd) <= 1e-6 * np.abs(g).max() + 1e-6, (i, g[i], fd)
