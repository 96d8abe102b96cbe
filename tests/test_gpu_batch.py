"""Batched persistent factorized CG over many uneven problems (one launch):
each problem's MLL and gradient match the single-problem path and the
oracle's estimator with the same probes."""
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


def problem(seed, d, m, n, nprobes, stats=torch.float32):
    rng = np.random.default_rng(seed)
    grid = oracle.make_grid(list(m), lo=0.0, hi=1.0)
    X = rng.uniform(0, 1, (d, n)).astype(np.float32)
    y = (np.sin(5 * X[0].astype(np.float64)) + 0.2 * rng.standard_normal(n)).astype(np.float32)
    xs = [torch.from_numpy(np.ascontiguousarray(X[k])).cuda() for k in range(d)]
    h = P.precompute(grid, xs, torch.from_numpy(y).cuda(), stats_dtype=stats,
                     n_probes=nprobes, probe_seed=100 + seed)
    hyp = {"lengthscale": [0.05 + 0.01 * seed] * d, "outputscale": 1.0 + 0.1 * seed,
           "noise": 0.2 + 0.02 * seed}
    return h, hyp, grid, X, y


def test_batch_matches_single_and_oracle():
    _need_gpu()
    specs = [(0, 1, [300], 20000, 9), (1, 2, [40, 33], 30000, 7), (2, 1, [1000], 50000, 15),
             (3, 2, [64, 64], 60000, 8), (4, 2, [20, 24], 5000, 3)]
    probs = [problem(*s) for s in specs]
    hs = [p[0] for p in probs]
    hyps = [p[1] for p in probs]
    mll_b, g_b, inf_b = P.batch_mll_and_grad(hs, hyps, lanczos_steps=10, tol=1e-10,
                                             maxiter=4000)
    for k, (h, hyp, grid, X, y) in enumerate(probs):
        mll_s, g_s, inf_s = P.mll_and_grad(h, hyp, lanczos_steps=10, tol=1e-10, maxiter=4000)
        scale = abs(inf_s["logdet"]) + abs(inf_s["quad"]) + h.n * math.log(2 * math.pi)
        assert abs(mll_b[k] - mll_s) <= 1e-7 * scale, (k, mll_b[k], mll_s)
        np.testing.assert_allclose(g_b[k], g_s, rtol=0, atol=1e-5 * np.max(np.abs(g_s)))
        assert inf_b[k]["iterations_probes_max"] > 0
    # one problem against the oracle's estimator with the same probes
    h, hyp, grid, X, y = probs[1]
    wtw, wty, yty = oracle.precompute(grid, X, y)
    sk = oracle.probe_sketches(grid, X, 101, 7)
    mll_o, g_o, inf_o = oracle.mll_and_grad(grid, hyp, wtw, wty, yty, X.shape[1], sk,
                                            lanczos_steps=10, tol=1e-10)
    scale = abs(inf_o["logdet"]) + abs(inf_o["q"]) + X.shape[1] * math.log(2 * math.pi)
    assert abs(mll_b[1] - mll_o) <= 1e-6 * scale
    np.testing.assert_allclose(g_b[1], g_o, rtol=0, atol=1e-4 * np.max(np.abs(g_o)))


def test_batch_deterministic_and_errors():
    _need_gpu()
    probs = [problem(5, 2, [30, 30], 8000, 5), problem(6, 1, [200], 4000, 4)]
    hs = [p[0] for p in probs]
    hyps = [p[1] for p in probs]
    a = P.batch_mll_and_grad(hs, hyps, 20, 1e-8, 2000)
    b = P.batch_mll_and_grad(hs, hyps, 20, 1e-8, 2000)
    assert a[0] == b[0] and a[1] == b[1]
    h3, hyp3, *_ = problem(7, 2, [20, 20], 1000, 0)
    with pytest.raises(P.FkgpError):
        P.batch_mll_and_grad(hs + [h3], hyps + [hyp3])
    # the batched passes take grid dimensions of at most 8192 nodes (the
    # standalone solver goes to 65536)
    h4, hyp4, *_ = problem(8, 1, [9000], 4000, 4)
    with pytest.raises(P.FkgpError, match="8192"):
        P.batch_mll_and_grad([h4], [hyp4])


def test_batch_bitwise_repeatable_across_regrouping():
    """The first evaluation of a batch groups right-hand sides by problem
    size alone; later ones also weigh the iterations each problem took, so a
    slow 2-D problem is split into smaller groups.  Every evaluation must
    still give bitwise the same values: a 2-D problem pairs only its own
    grid lines in the complex FFTs (41 lines per vector: one half-empty
    pair), a 1-D problem keeps the size-based groups."""
    _need_gpu()
    probs = [problem(21, 1, [4000], 30000, 7), problem(22, 2, [41, 41], 20000, 7),
             problem(23, 2, [25, 33], 5000, 5)]
    hs = [p[0] for p in probs]
    hyps = [p[1] for p in probs]
    hyps[0].update(lengthscale=[0.2], noise=0.5)
    hyps[1].update(lengthscale=[0.02, 0.02], noise=0.01)
    runs = [P.batch_mll_and_grad(hs, hyps, 20, 1e-8, 3000) for _ in range(3)]
    its = [i["iterations_probes_max"] for i in runs[0][2]]
    assert its[1] > 5 * its[0], its   # the regrouping case is exercised
    for m, g, _ in runs[1:]:
        assert m == runs[0][0]
        assert g == runs[0][1]


def test_batch_toeplitz_path_limits():
    """2-D problems at the limits of the dense Toeplitz line passes: 128 x 128
    (largest on that path), 129 x 40 (line FFT: one dimension too long), and
    65 x 7 (two 64-row blocks, lines shorter than one 8-output block); each
    matches the single-problem path."""
    _need_gpu()
    specs = [(31, 2, [128, 128], 30000, 3), (32, 2, [129, 40], 20000, 3),
             (33, 2, [65, 7], 6000, 3)]
    probs = [problem(*s) for s in specs]
    hs = [p[0] for p in probs]
    hyps = [p[1] for p in probs]
    # 10 Lanczos steps as in the other batch-vs-single comparisons (the
    # coefficients come from CG and carry its rounding into the estimate)
    mll_b, g_b, inf_b = P.batch_mll_and_grad(hs, hyps, lanczos_steps=10, tol=1e-10,
                                             maxiter=20000)
    for k, h in enumerate(hs):
        mll_s, g_s, inf_s = P.mll_and_grad(h, hyps[k], 10, 1e-10, 20000)
        assert inf_b[k]["status"] == 0 and inf_s["status"] == 0
        print(f"{k}: logdet {inf_b[k]['logdet']:.12g} / {inf_s['logdet']:.12g}, quad "
              f"{inf_b[k]['quad']:.12g} / {inf_s['quad']:.12g}")
        scale = abs(inf_s["logdet"]) + abs(inf_s["quad"]) + h.n * math.log(2 * math.pi)
        assert abs(mll_b[k] - mll_s) <= 1e-7 * scale, (k, mll_b[k], mll_s)
        np.testing.assert_allclose(g_b[k], g_s, rtol=0, atol=1e-5 * np.max(np.abs(g_s)))


def test_batch_long_lines():
    """1-D problems with 1500 .. 8192 nodes (circulants of 4096 .. 16384
    points, four-step line FFT inside the persistent kernel) beside short
    ones; each matches the single-problem path, one matches the oracle."""
    _need_gpu()
    specs = [(8, 1, [1500], 20000, 5), (9, 1, [3000], 40000, 9), (10, 1, [8192], 60000, 4),
             (11, 2, [2100, 12], 30000, 6), (12, 2, [30, 30], 8000, 3)]
    probs = [problem(*s) for s in specs]
    hs = [p[0] for p in probs]
    hyps = [p[1] for p in probs]
    for hyp in hyps[:4]:
        hyp["lengthscale"][0] = 0.004
    mll_b, g_b, inf_b = P.batch_mll_and_grad(hs, hyps, lanczos_steps=10, tol=1e-10,
                                             maxiter=8000)
    for k, (h, hyp, grid, X, y) in enumerate(probs):
        mll_s, g_s, inf_s = P.mll_and_grad(h, hyp, lanczos_steps=10, tol=1e-10, maxiter=8000)
        scale = abs(inf_s["logdet"]) + abs(inf_s["quad"]) + h.n * math.log(2 * math.pi)
        assert abs(mll_b[k] - mll_s) <= 1e-7 * scale, (k, mll_b[k], mll_s)
        np.testing.assert_allclose(g_b[k], g_s, rtol=0, atol=1e-5 * np.max(np.abs(g_s)))
    h, hyp, grid, X, y = probs[1]
    wtw, wty, yty = oracle.precompute(grid, X, y)
    sk = oracle.probe_sketches(grid, X, 109, 9)
    mll_o, g_o, inf_o = oracle.mll_and_grad(grid, hyp, wtw, wty, yty, X.shape[1], sk,
                                            lanczos_steps=10, tol=1e-10)
    scale = abs(inf_o["logdet"]) + abs(inf_o["q"]) + X.shape[1] * math.log(2 * math.pi)
    assert abs(mll_b[1] - mll_o) <= 1e-6 * scale
    np.testing.assert_allclose(g_b[1], g_o, rtol=0, atol=1e-4 * np.max(np.abs(g_o)))


def test_batch_tiles_agree_and_autotune():
    """Every (right-hand sides per workgroup, workgroup size) tile gives the
    same result up to rounding (the workgroup size changes the reduction
    order and, for 1-D problems, the grouping changes which right-hand sides
    share a complex FFT, and Lanczos coefficients taken from CG pass rounding
    on, so the comparison uses the batch-vs-single tolerance); at one
    workgroup size a 2-D problem gives bitwise the same values for every
    group size, since its grid lines are paired within one right-hand side;
    the autotuner reports the tile it chose."""
    _need_gpu()
    probs = [problem(13, 2, [45, 37], 20000, 6), problem(14, 1, [700], 15000, 9),
             problem(15, 2, [20, 70], 9000, 4)]
    hs = [p[0] for p in probs]
    hyps = [p[1] for p in probs]
    for hyp in hyps:
        hyp["lengthscale"] = [0.05] * len(hyp["lengthscale"])
    ref = {}
    for nr in (2, 4, 8):
        for block in (256, 512):
            m, g, inf = P.batch_mll_and_grad(hs, hyps, 10, 1e-9, 4000, batch_rhs=nr,
                                             batch_block=block)
            assert all(i["batch_rhs"] == nr and i["batch_block"] == block for i in inf)
            if block not in ref:
                ref[block] = (m, g, inf)
                if block == 256:
                    continue
            else:
                for k in (0, 2):   # the 2-D problems
                    assert m[k] == ref[block][0][k] and g[k] == ref[block][1][k], (nr, block, k)
            r0 = ref[256]
            for k in range(len(hs)):
                scale = (abs(r0[2][k]["logdet"]) + abs(r0[2][k]["quad"])
                         + hs[k].n * math.log(2 * math.pi))
                assert abs(m[k] - r0[0][k]) <= 1e-7 * scale, (nr, block, k)
                np.testing.assert_allclose(g[k], r0[1][k], rtol=0,
                                           atol=1e-5 * np.max(np.abs(r0[1][k])))
    m, g, inf = P.batch_mll_and_grad(hs, hyps, 10, 1e-9, 4000)
    assert inf[0]["batch_rhs"] in (2, 4, 8) and inf[0]["batch_block"] in (256, 512)
    with pytest.raises(P.FkgpError):
        P.batch_mll_and_grad(hs, hyps, 10, 1e-9, 4000, batch_rhs=3)


def test_batch64_workload_subset():
    """Problems of the many-problem workload (1-D lines of 512 .. 8192 nodes,
    2-D grids of 32^2 .. 128^2, 32 right-hand sides each) at reduced n: the
    one-launch result matches the per-problem path."""
    _need_gpu()
    from paper_2101_11751_amd import workloads
    wl = workloads.batch64(device=torch.device("cuda"), n_scale=0.02,
                           which=[0, 4, 6, 30, 32, 36, 45, 59])
    hs = [P.precompute(w["grid"], w["x"], w["y"], stats_dtype=torch.float32,
                       n_probes=w["nprobes"], probe_seed=w["probe_seed"]) for w in wl]
    hyps = [w["hypers"] for w in wl]
    mb, gb, ib = P.batch_mll_and_grad(hs, hyps, 30, 1e-8, 20000)
    for k, h in enumerate(hs):
        ms, gs, inf = P.mll_and_grad(h, hyps[k], 30, 1e-8, 20000)
        assert inf["status"] == 0 and ib[k]["status"] == 0
        scale = abs(inf["logdet"]) + abs(inf["quad"]) + h.n * math.log(2 * math.pi)
        print(f"{k}: m={h.m_total} n={h.n}: mll {mb[k]:.12g} / {ms:.12g}, logdet "
              f"{ib[k]['logdet']:.12g} / {inf['logdet']:.12g}, quad {ib[k]['quad']:.12g} / "
              f"{inf['quad']:.12g}, iterations y {ib[k]['iterations_y']} / "
              f"{inf['iterations_y']}, probes {ib[k]['iterations_probes_max']} / "
              f"{inf['iterations_probes_max']}")
        assert abs(mb[k] - ms) <= 1e-6 * scale, (k, mb[k], ms)
        np.testing.assert_allclose(gb[k], gs, rtol=0, atol=1e-4 * np.max(np.abs(gs)))


def test_batch_response_norm_not_n():
    """The data right-hand side enters the factorized inner products with
    ||y||^2 = y^T y, the probes with n: a response scaled far from unit
    variance (y^T y = 400 n here) must give the single-problem result."""
    _need_gpu()
    rng = np.random.default_rng(16)
    n = 6000
    grid = oracle.make_grid([50, 40], lo=0.0, hi=1.0)
    X = rng.uniform(0, 1, (2, n)).astype(np.float32)
    y = (20.0 * np.sign(np.sin(7 * X[0].astype(np.float64)))
         + rng.standard_normal(n)).astype(np.float32)
    xs = [torch.from_numpy(np.ascontiguousarray(X[k])).cuda() for k in range(2)]
    h = P.precompute(grid, xs, torch.from_numpy(y).cuda(), stats_dtype=torch.float32,
                     n_probes=5, probe_seed=7)
    hyp = {"lengthscale": [0.06, 0.06], "outputscale": 50.0, "noise": 1.0}
    mb, gb, ib = P.batch_mll_and_grad([h], [hyp], 10, 1e-10, 5000)
    ms, gs, inf = P.mll_and_grad(h, hyp, 10, 1e-10, 5000)
    assert ib[0]["iterations_y"] > 5
    assert abs(ib[0]["quad"] - inf["quad"]) <= 1e-6 * inf["quad"]
    scale = abs(inf["logdet"]) + abs(inf["quad"]) + n * math.log(2 * math.pi)
    assert abs(mb[0] - ms) <= 1e-7 * scale


def test_batch64_long_1d_against_oracle():
    """Long 1-D problems of the many-problem workload (4,365 and 7,549
    nodes, lengthscales of ~100 and ~245 nodes, four-step line FFTs) with 30
    Lanczos steps: both GPU paths against the oracle's estimator with the
    same probes (the oracle's own log-determinant moves by ~3e-11 when only
    the rounding of K_G changes, FFT or dense)."""
    _need_gpu()
    from paper_2101_11751_amd import workloads
    wls = workloads.batch64(device="cpu", n_scale=0.02, which=[4, 30])
    hs, hyps, data = [], [], []
    for w in wls:
        X = np.stack([x.numpy() for x in w["x"]])
        y = w["y"].numpy()
        xs = [torch.from_numpy(np.ascontiguousarray(X[k])).cuda() for k in range(X.shape[0])]
        hs.append(P.precompute(w["grid"], xs, torch.from_numpy(y).cuda(),
                               stats_dtype=torch.float64, n_probes=w["nprobes"],
                               probe_seed=w["probe_seed"]))
        hyps.append(w["hypers"])
        data.append((X, y))
    tol = 1e-10
    mb, gb, ib = P.batch_mll_and_grad(hs, hyps, 30, tol, 20000)
    for k, w in enumerate(wls):
        X, y = data[k]
        ms, gs, inf = P.mll_and_grad(hs[k], hyps[k], 30, tol, 20000)
        wtw, wty, yty = oracle.precompute(w["grid"], X, y)
        sk = oracle.probe_sketches(w["grid"], X, w["probe_seed"], w["nprobes"])
        mo, go, io = oracle.mll_and_grad(w["grid"], hyps[k], wtw, wty, yty, X.shape[1], sk,
                                         lanczos_steps=30, tol=tol, maxiter=20000)
        print(f"{w['name']} m={w['grid']['m']}: logdet batch {ib[k]['logdet']:.12g} single "
              f"{inf['logdet']:.12g} oracle {io['logdet']:.12g}; quad batch "
              f"{ib[k]['quad']:.12g} single {inf['quad']:.12g} oracle {io['q']:.12g}; "
              f"probe iterations batch {ib[k]['iterations_probes_max']} single "
              f"{inf['iterations_probes_max']}")
        q_bound = 2 * tol * yty / hyps[k]["noise"] ** 2
        for name, ld, q in (("batch", ib[k]["logdet"], ib[k]["quad"]),
                            ("single", inf["logdet"], inf["quad"])):
            assert abs(ld - io["logdet"]) <= 1e-9 * abs(io["logdet"]), name
            assert abs(q - io["q"]) <= 1e-9 * abs(io["q"]) + q_bound, name
