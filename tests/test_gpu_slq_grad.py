"""Gradient of the stochastic Lanczos log-determinant estimate itself
(trace_mode 2: reverse mode through each probe's Lanczos steps, the
checkpointed Krylov vectors being the factorized CG's residuals; Sec. 2.1
and the appendix's factorized Lanczos): against the oracle's reverse sweep
on small grids (d = 1, 2, 3), and against central differences of the
returned estimate on the full differentiation workload."""
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


def shifted(hyp, i, d, e):
    hp = {"lengthscale": list(hyp["lengthscale"]), "outputscale": hyp["outputscale"],
          "noise": hyp["noise"]}
    f = math.exp(e)
    if i < d:
        hp["lengthscale"][i] *= f
    elif i == d:
        hp["outputscale"] *= f
    else:
        hp["noise"] *= f
    return hp


@pytest.mark.parametrize("m,n,steps", [([200], 3000, 12), ([30, 25], 5000, 15),
                                       ([10, 9, 8], 3000, 10)])
def test_slq_gradient_matches_oracle(m, n, steps):
    _need_gpu()
    d = len(m)
    rng = np.random.default_rng(70 + d)
    grid = oracle.make_grid(m, lo=0.0, hi=1.0)
    X = rng.uniform(0, 1, (d, n))
    y = np.sin(5 * X[0]) + 0.2 * rng.standard_normal(n)
    hyp = {"lengthscale": [0.12] * d, "outputscale": 1.3, "noise": 0.25}
    nprobes, seed = 4, 11
    xs = [torch.from_numpy(np.ascontiguousarray(X[k])).cuda() for k in range(d)]
    h = P.precompute(grid, xs, torch.from_numpy(y).cuda(), stats_dtype=torch.float64,
                     n_probes=nprobes, probe_seed=seed)
    mll, g, inf = P.mll_and_grad(h, hyp, lanczos_steps=steps, tol=1e-12, maxiter=20000,
                                 trace="slq")
    wtw, wty, yty = oracle.precompute(grid, X, y)
    sk = oracle.probe_sketches(grid, X, seed, nprobes)
    mo, go, io = oracle.mll_and_grad(grid, hyp, wtw, wty, yty, n, sk, lanczos_steps=steps,
                                     tol=1e-12, maxiter=20000, slq_grad=True)
    print(f"d={d}: grad {np.array(g)}, oracle {go}")
    assert abs(inf["logdet"] - io["logdet"]) <= 1e-10 * abs(io["logdet"])
    np.testing.assert_allclose(g, go, rtol=0, atol=1e-8 * np.max(np.abs(go)))
    # the Hutchinson gradient is a different quantity (an estimate of the
    # trace, not the derivative of the estimate)
    _, gh, _ = P.mll_and_grad(h, hyp, lanczos_steps=steps, tol=1e-12, maxiter=20000)
    assert np.max(np.abs(np.array(gh) - np.array(g))) > 1e-6 * np.max(np.abs(go))


@pytest.mark.slow
def test_slq_gradient_finite_differences_full_size():
    """Differentiation workload (n = 4e6, 256^2, 16 probes, 30 Lanczos steps,
    offset hyperparameters): central differences of the returned
    log-determinant estimate against the log-determinant part of the
    trace_mode-2 gradient, tr = -dquad - 2 grad.  At 30 steps the estimate
    is strongly curved in theta (the h^2 term of a central difference with
    h = 1e-4 is ~7e-4 of the derivative, falling 100x per 10x in h), so
    the differences at h = 1e-4 and h/2 are combined by one Richardson step,
    (4 D(h/2) - D(h)) / 3, which removes it."""
    _need_gpu()
    from paper_2101_11751_amd import workloads
    wl = workloads.prior2d()
    hyp = wl["hypers_offset"]
    h = P.precompute(wl["grid"], [x.cuda() for x in wl["x"]], wl["y"].cuda(),
                     stats_dtype=torch.float32, n_probes=wl["nprobes"],
                     probe_seed=wl["probe_seed"])
    steps, tol = 30, 1e-10
    _, g, inf = P.mll_and_grad(h, hyp, lanczos_steps=steps, tol=tol, maxiter=100000,
                               trace="slq")
    tr = -np.array(inf["dquad"][:4]) - 2.0 * np.array(g)

    def logdet(hp):
        return P.mll_and_grad(h, hp, lanczos_steps=steps, tol=tol, maxiter=100000)[2]["logdet"]

    eps = 1e-4
    for i in range(4):
        fd = [(logdet(shifted(hyp, i, 2, e)) - logdet(shifted(hyp, i, 2, -e))) / (2 * e)
              for e in (eps, eps / 2)]
        rich = (4.0 * fd[1] - fd[0]) / 3.0
        print(f"dlogdet/dtheta_{i}: reverse mode {tr[i]:.10g}, central differences "
              f"{fd[0]:.10g} (h = 1e-4), extrapolated {rich:.10g}")
        assert abs(rich - tr[i]) <= 1e-5 * abs(tr[i]), (i, rich, tr[i])
