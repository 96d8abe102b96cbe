#!/usr/bin/env python
"""Benchmark of the fkgp hot path on one MI355X; prints ONE JSON line.

A step is one pass of the hot path over the 3-D sweep-shaped workload
(n = 1e8 points in a cylinder, m = 100 x 100 x 30 = 300,000 grid nodes, FP32
inputs, W^T W stored in FP32): the one-shot O(n) precompute of W^T W, W^T y,
y^T y followed by the posterior-mean solve (spectra, the simplified
factorized CG with FP64 operator arithmetic on the FP32-stored W^T W and FP64
vectors and scalars, final K_G product).  Inputs are generated on the device
before timing.

value            = n * steps / timed seconds  (Mpts/s through the whole step)
mll_grad         = differentiation workload: batched FP32 vs plain FP64 path
batch_mll_grad   = many-problem workload: one persistent launch vs a loop
ski_sweep        = per-iteration time, factorized CG vs the plain SKI CG in
                   n-space, on the synthetic sine with m = n, n/16, sqrt(n)
precompute_*     = n / precompute time (precompute_host: from host memory,
                   PCIe transfers included)
cg_mvms_per_s    = CG iterations (one operator B each) per second of solve
roofline         = banded W^T W product as the CG loop launches it (with its
                   fused u^T r reduction), algorithmic bytes / average launch
                   duration (HIP events on the library's stream, hot); the
                   algorithmic bytes are the exact nonzero entries of W^T W
                   (FP32) plus x and u (FP64); the fraction on the nonzero
                   64-row blocks (what the kernel reads) and a cold figure
                   (512 MiB written between launches) are reported beside it
mean_rel_err_vs_f64_tight = the timed solve's mu_G against an FP64-statistics
                   solve to relative residual 1e-8 on the same points
cpu_baseline     = the FP64 CPU oracle on a bounded sample, scaled to the
                   same per-step work (see "sample"), on all host cores
                   (OpenMP statistics and product, threaded FFTs) and on one
"""
import argparse
import json
import math
import os
import sys
import time

HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of the banded product on this workload, from the two
# rocprofv3 --pmc runs (FETCH_SIZE x 1.9997, WRITE_SIZE x 1.0, calibrated on a
# 256 MiB copy) recorded in profiles/radar3d_hbm_traffic_pmc.md.  Set to None
# whenever spmv_tiled_kernel changes until the counters are taken again.
SPMV_TRAFFIC_BYTES = 340.9e6


def _parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=100_000_000)
    ap.add_argument("--tol", type=float, default=1e-2)
    ap.add_argument("--maxiter", type=int, default=20000)
    ap.add_argument("--mvm-reps", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-mll", action="store_true")
    ap.add_argument("--mll-reps", type=int, default=2)
    ap.add_argument("--mll-tol", type=float, default=1e-4)
    ap.add_argument("--mll-maxiter", type=int, default=20000)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-batch-loop", action="store_true",
                    help="batch64 without the per-problem comparison loop (profiling runs)")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-cov", action="store_true")
    ap.add_argument("--batch-tol", type=float, default=1e-4)
    ap.add_argument("--batch-maxiter", type=int, default=30000)
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def host_cpu():
    """CPU model and the number of cores this process may run on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return model, avail


def cpu_baseline(wl, n_total, iters, budget_s):
    """Times the oracle (FP64 C statistics + NumPy/SciPy operator) on a
    bounded sample and scales it to one step of the full workload: on all
    the cores this process may use (OpenMP statistics with per-thread
    accumulators combined in thread order, row-parallel banded product,
    threaded FFTs) and on one core (the serial reference)."""
    import numpy as np
    import oracle
    grid = wl["grid"]
    model, avail = host_cpu()
    threads = max(1, min(avail, int(os.environ.get("OMP_NUM_THREADS", avail))))
    out = {}
    for name, th, share in (("all", threads, 0.6), ("one", 1, 0.25)):
        # precompute: calibrate on a small sample, then size it to the budget
        n_cal = 20_000 * th
        xs = [c[:n_cal].cpu().numpy() for c in wl["x"]]
        ys = wl["y"][:n_cal].cpu().numpy()
        t0 = time.perf_counter()
        oracle.precompute(grid, xs, ys, threads=th)
        per_pt = (time.perf_counter() - t0) / n_cal
        n_s = int(min(n_total, max(n_cal, share * budget_s / per_pt)))
        xs = [c[:n_s].cpu().numpy() for c in wl["x"]]
        ys = wl["y"][:n_s].cpu().numpy()
        t0 = time.perf_counter()
        wtw, wty, yty = oracle.precompute(grid, xs, ys, threads=th)
        t_pre = time.perf_counter() - t0
        # operator B at the full grid size (the oracle's MVM), 2 reps
        v = np.random.default_rng(0).standard_normal(wty.shape[0])
        reps = 2
        t0 = time.perf_counter()
        for _ in range(reps):
            oracle.B_apply(grid, wl["hypers"], wtw, v, threads=th)
        t_mvm = (time.perf_counter() - t0) / reps
        t_step = t_pre * (n_total / n_s) + iters * t_mvm
        out[name] = {"value": n_total / t_step / 1e6, "threads": th, "n_sample": n_s,
                     "precompute_s": t_pre, "precompute_mpts_per_s": n_s / t_pre / 1e6,
                     "mvm_s": t_mvm, "mvm_per_s": 1.0 / t_mvm}
        log(f"cpu oracle, {th} thread(s): precompute {n_s / t_pre / 1e6:.4f} Mpts/s on {n_s} "
            f"points, operator {1.0 / t_mvm:.2f} MVM/s, scaled step {out[name]['value']:.5f} Mpts/s")
        del wtw, wty
    a, o = out["all"], out["one"]
    return {"value": a["value"], "unit": "Mpts/s", "cores": a["threads"], "kind": "oracle",
            "cpu": model, "cores_available": avail,
            "sample": (f"oracle statistics on the first {a['n_sample']} points "
                       f"({a['precompute_s']:.1f} s, {a['precompute_mpts_per_s']:.4f} Mpts/s on "
                       f"{a['threads']} threads) scaled to n={n_total}, plus {iters:.0f} oracle "
                       f"operator applications at m={int(np.prod(grid['m']))} "
                       f"({a['mvm_s']:.3f} s each, 2 timed)"),
            "precompute_mpts_per_s": a["precompute_mpts_per_s"], "mvm_per_s": a["mvm_per_s"],
            "one_core": {"value": o["value"], "precompute_mpts_per_s": o["precompute_mpts_per_s"],
                         "mvm_per_s": o["mvm_per_s"], "n_sample": o["n_sample"]}}


def mll_compare(P, workloads, torch, dev, reps, tol, maxiter):
    """MLL + gradient on the differentiation workload (n=4e6, 256x256 grid,
    16 Rademacher probes, 30 Lanczos steps) at the offset hyperparameters:
    batched probes on FP32-stored statistics vs one-probe-at-a-time on FP64
    statistics (the plain FP64 path), both with FP64 CG scalars."""
    wl = workloads.prior2d(device=dev)
    torch.cuda.synchronize()
    hyp = wl["hypers_offset"]
    out = {}
    for name, sdt, batched in (("batched_f32", torch.float32, True),
                               ("plain_f64", torch.float64, False)):
        h = P.precompute(wl["grid"], wl["x"], wl["y"], stats_dtype=sdt,
                         n_probes=wl["nprobes"], probe_seed=wl["probe_seed"])
        P.mll_and_grad(h, hyp, wl["lanczos_steps"], tol, maxiter, batched=batched)  # warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            val, g, info = P.mll_and_grad(h, hyp, wl["lanczos_steps"], tol, maxiter,
                                          batched=batched)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        out[name] = {"s_per_eval": dt, "mll": val, "grad": g, "status": info["status"],
                     "iterations_y": info["iterations_y"],
                     "iterations_probes_max": info["iterations_probes_max"]}
        log(f"mll {name}: {dt:.3f} s/eval, mll={val:.6f}, iters y={info['iterations_y']} "
            f"probes={info['iterations_probes_max']}")
        h.close()
    a, b = out["batched_f32"], out["plain_f64"]
    import numpy as np
    gdiff = float(np.max(np.abs(np.array(a["grad"]) - np.array(b["grad"])))
                  / np.max(np.abs(np.array(b["grad"]))))
    # accuracy of both timed paths against a tight FP64 reference with the
    # same probes and Lanczos size (FP64 statistics, solves to 1e-10)
    h = P.precompute(wl["grid"], wl["x"], wl["y"], stats_dtype=torch.float64,
                     n_probes=wl["nprobes"], probe_seed=wl["probe_seed"])
    ref_tol = 1e-10
    rv, rg, ri = P.mll_and_grad(h, hyp, wl["lanczos_steps"], ref_tol, 200000, batched=True)
    h.close()
    rg = np.array(rg)
    for rec in (a, b):
        rec["mll_rel_err_vs_ref"] = abs(rec["mll"] - rv) / abs(rv)
        rec["grad_rel_err_vs_ref"] = float(np.max(np.abs(np.array(rec["grad"]) - rg))
                                           / np.max(np.abs(rg)))
    log(f"mll reference (FP64, tol {ref_tol:g}): {rv:.6f}; errors: batched FP32 "
        f"{a['mll_rel_err_vs_ref']:.2e} / {a['grad_rel_err_vs_ref']:.2e}, plain FP64 "
        f"{b['mll_rel_err_vs_ref']:.2e} / {b['grad_rel_err_vs_ref']:.2e}")
    return {"workload": "prior2d: n=4e6 x~U[0,1]^2, grid 256x256, GSGP-prior y (l=0.04, "
                        "s=1.5, sigma=0.1), evaluated at l=0.05, s=1.0, sigma=0.15; 16 probes, "
                        "30 Lanczos steps, tol %g" % tol,
            "batched_f32_s_per_eval": a["s_per_eval"], "plain_f64_s_per_eval": b["s_per_eval"],
            "speedup": b["s_per_eval"] / a["s_per_eval"],
            "mll_rel_diff": abs(a["mll"] - b["mll"]) / abs(b["mll"]), "grad_rel_diff": gdiff,
            "reference": {"stats": "f64", "tol": ref_tol, "mll": rv, "grad": rg.tolist(),
                          "iterations_y": ri["iterations_y"],
                          "iterations_probes_max": ri["iterations_probes_max"]},
            "batched_f32_mll_rel_err": a["mll_rel_err_vs_ref"],
            "batched_f32_grad_rel_err": a["grad_rel_err_vs_ref"],
            "plain_f64_mll_rel_err": b["mll_rel_err_vs_ref"],
            "plain_f64_grad_rel_err": b["grad_rel_err_vs_ref"],
            "mll": b["mll"], "grad": b["grad"],
            "converged": a["status"] == 0 and b["status"] == 0,
            "iterations_y": b["iterations_y"], "iterations_probes_max": b["iterations_probes_max"]}


def batch_compare(P, workloads, torch, dev, tol, maxiter, loop_cmp=True):
    """The many-problem workload (64 uneven problems, 32 right-hand sides
    each): MLL + gradient of every problem in one persistent launch (tiles
    autotuned; the tuning trial runs in an untimed first call) vs one
    mll_and_grad call per problem (probes batched within each problem), both
    on FP32-stored statistics with FP64 vectors and scalars."""
    import numpy as np
    probs = workloads.batch64(device=dev)
    torch.cuda.synchronize()
    n_total = sum(p["n"] for p in probs)
    t0 = time.perf_counter()
    hs = [P.precompute(p["grid"], p["x"], p["y"], stats_dtype=torch.float32,
                       n_probes=p["nprobes"], probe_seed=p["probe_seed"]) for p in probs]
    torch.cuda.synchronize()
    t_pre = time.perf_counter() - t0
    hyps = [p["hypers"] for p in probs]
    steps = probs[0]["lanczos_steps"]
    P.batch_mll_and_grad(hs, hyps, steps, tol, maxiter)   # tile autotuning + warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mb, gb, ib = P.batch_mll_and_grad(hs, hyps, steps, tol, maxiter)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    log(f"batch64: one launch {t_batch:.3f} s (tile {ib[0]['batch_rhs']} rhs x "
        f"{ib[0]['batch_block']} threads)")
    if not loop_cmp:
        iters = max(max(i["iterations_y"], i["iterations_probes_max"]) for i in ib)
        for h in hs:
            h.close()
        return {"workload": "batch64 (one launch only)", "n_total": n_total,
                "batched_s_per_eval": t_batch, "iterations_max": iters}
    t0 = time.perf_counter()
    loop = [P.mll_and_grad(h, hyp, steps, tol, maxiter) for h, hyp in zip(hs, hyps)]
    torch.cuda.synchronize()
    t_loop = time.perf_counter() - t0
    log(f"batch64: per-problem loop {t_loop:.3f} s")
    rel_mll = max(abs(a - l[0]) / abs(l[0]) for a, l in zip(mb, loop))
    rel_q = max(abs(i["quad"] - l[2]["quad"]) / abs(l[2]["quad"]) for i, l in zip(ib, loop))
    rel_g = max(float(np.max(np.abs(np.array(g) - np.array(l[1]))) / np.max(np.abs(l[1])))
                for g, l in zip(gb, loop))
    conv = all(i["status"] == 0 for i in ib) and all(l[2]["status"] == 0 for l in loop)
    for h in hs:
        h.close()
    return {"workload": "batch64: 32 1-D (m 512..8192, n 1e4..2e6, sine data) + 32 2-D "
                        "(m 32^2..128^2, n 5e4..1e6, bump data) problems, l~U[0.01,0.1], "
                        "31 probes + y per problem, %d Lanczos steps, tol %g" % (steps, tol),
            "n_total": n_total, "precompute_s": t_pre,
            "batched_s_per_eval": t_batch, "per_problem_loop_s_per_eval": t_loop,
            "speedup": t_loop / t_batch,
            "tile": {"rhs_per_workgroup": ib[0]["batch_rhs"],
                     "threads_per_workgroup": ib[0]["batch_block"]},
            "iterations_max": max(max(i["iterations_y"], i["iterations_probes_max"]) for i in ib),
            "max_rel_diff_mll": rel_mll, "max_rel_diff_quad": rel_q, "max_rel_diff_grad": rel_g,
            "converged": conv}


def precompute_extra(P, workloads, torch, dev, reps=3):
    """Precompute throughput on the 2-D bump workload (128x128 grid) at
    n = 1e6 (its own size) and n = 1e8 (large enough for a bandwidth
    figure): Mpts/s of the best of `reps` timed calls after a warm-up."""
    out = {}
    for n in (1_000_000, 100_000_000):
        wl = workloads.bumps2d(n=n, device=dev)
        torch.cuda.synchronize()
        best = None
        for r in range(reps + 1):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            h = P.precompute(wl["grid"], wl["x"], wl["y"], stats_dtype=torch.float32)
            e1.record()
            torch.cuda.synchronize()
            t = e0.elapsed_time(e1) / 1e3
            if r > 0:
                best = t if best is None else min(best, t)
            h.close()
        out[f"bumps2d_n{n:.0e}".replace("+0", "")] = {"ms": best * 1e3, "mpts_per_s": n / best / 1e6}
        log(f"precompute bumps2d n={n}: {best*1e3:.2f} ms, {n/best/1e6:.0f} Mpts/s")
        del wl
        torch.cuda.empty_cache()
    return out


def precompute_host_leg(P, torch, wl, n, reps=2):
    """The main workload's precompute from points in host memory (pageable
    arrays streamed in chunks of 2^24 points through pinned staging): the
    PCIe-inclusive rate, best of `reps` after a warm-up."""
    xs = [t.cpu().numpy() for t in wl["x"]]
    y = wl["y"].cpu().numpy()
    best = None
    for r in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = P.precompute_host(wl["grid"], xs, y, stats_dtype=torch.float32)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        h.close()
        if r > 0:
            best = t if best is None else min(best, t)
    log(f"precompute from host memory: {best*1e3:.1f} ms, {n/best/1e6:.0f} Mpts/s")
    return {"ms": best * 1e3, "mpts_per_s": n / best / 1e6, "chunk": 1 << 24,
            "note": "pageable host arrays, pinned staging, copies on a second stream"}


def ski_sweep(P, workloads, torch, dev, iters=200):
    """Per-iteration time of the factorized CG (operator on m grid nodes,
    independent of n) and of the plain SKI CG (n-space, O(n + m log m) per
    iteration) on the synthetic sine with m = n, n/16 and sqrt(n): the
    paper's per-iteration comparison (Sec. 5, Fig. 2).  Each solve runs
    exactly `iters` iterations (tol 0) after a short warm-up; the time per
    iteration includes each solver's set-up, amortised over the iterations."""
    cases = [(1024, "n"), (4096, "n"), (8192, "n"), (32768, "n"), (65536, "n"),
             (16384, "n/16"), (65536, "n/16"), (131072, "n/16"), (1_048_576, "n/16"),
             (10_000, "sqrt(n)"), (1_000_000, "sqrt(n)"), (64_000_000, "sqrt(n)")]
    out = []
    for n, rule in cases:
        m = n if rule == "n" else (n // 16 if rule == "n/16" else int(round(math.sqrt(n))))
        wl = workloads.sine1d_grid(n, m, device=dev)
        h = P.precompute(wl["grid"], wl["x"], wl["y"], stats_dtype=torch.float64,
                         keep_points=True)
        hyp = wl["hypers"]
        P.solve(h, hyp, tol=0.0, maxiter=5)
        P.ski_solve(h, hyp, tol=0.0, maxiter=5)
        rec = {"n": n, "m": m, "rule": rule}
        for name, fn in (("gsgp", P.solve), ("ski", P.ski_solve)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, info = fn(h, hyp, tol=0.0, maxiter=iters)
            torch.cuda.synchronize()
            rec[f"{name}_us_per_iter"] = (time.perf_counter() - t0) / max(info["iterations"], 1) * 1e6
        rec["ski_over_gsgp"] = rec["ski_us_per_iter"] / rec["gsgp_us_per_iter"]
        log(f"sweep n={n} m={m} ({rule}): gsgp {rec['gsgp_us_per_iter']:.1f} us/it, "
            f"ski {rec['ski_us_per_iter']:.1f} us/it")
        out.append(rec)
        h.close()
        del wl
        torch.cuda.empty_cache()
    return out


def radar_iter_leg(P, workloads, torch, dev, iters=200):
    """Per-iteration time of the factorized CG and of the plain SKI CG on the
    radar-shaped 3-D workload at the size of the paper's per-iteration
    comparison on radar data (Table 1: n = 10.5M, m = 51.2K = 40 x 40 x 32);
    each solve runs exactly `iters` iterations after a short warm-up."""
    wl = workloads.radar3d(n=10_500_000, device=dev, m=(40, 40, 32))
    h = P.precompute(wl["grid"], wl["x"], wl["y"], stats_dtype=torch.float64, keep_points=True)
    hyp = wl["hypers"]
    P.solve(h, hyp, tol=0.0, maxiter=5)
    P.ski_solve(h, hyp, tol=0.0, maxiter=5)
    rec = {"n": 10_500_000, "m": 51200, "grid": [40, 40, 32]}
    for name, fn in (("gsgp", P.solve), ("ski", P.ski_solve)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info = fn(h, hyp, tol=0.0, maxiter=iters)
        torch.cuda.synchronize()
        rec[f"{name}_us_per_iter"] = (time.perf_counter() - t0) / max(info["iterations"], 1) * 1e6
    rec["gsgp_over_ski"] = rec["gsgp_us_per_iter"] / rec["ski_us_per_iter"]
    log(f"radar n=10.5M m=51.2K: gsgp {rec['gsgp_us_per_iter']:.1f} us/it, "
        f"ski {rec['ski_us_per_iter']:.1f} us/it (ratio {rec['gsgp_over_ski']:.4f})")
    h.close()
    del wl
    torch.cuda.empty_cache()
    return rec


def cov_leg(P, workloads, torch, dev, nq=691, tol=1e-10, maxiter=20000):
    """Exact SKI posterior covariance between nq query points (one solve per
    query point; Sec. 5 computes a 691 x 691 matrix on the sound data, n =
    59.3K) on the synthetic sine of the same size, for a small and a large
    grid (m = 1000, 8000 and 60000, the paper's largest sound grid): seconds
    per call after a warm-up; then the rank-k covariance (k = min(m, 10000)) built from the
    factorized Lanczos, its build and query times and its relative Frobenius
    distance from the exact matrix."""
    out = []
    g = torch.Generator(device=dev)
    g.manual_seed(5)
    xq = torch.rand(nq, generator=g, device=dev, dtype=torch.float64)
    for m in (1000, 8000, 60000):
        wl = workloads.sine1d_grid(59_300, m, device=dev)
        h = P.precompute(wl["grid"], wl["x"], wl["y"], stats_dtype=torch.float64)
        hyp = wl["hypers"]
        P.posterior_cov(h, hyp, [xq[:64]], tol=tol, maxiter=maxiter)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        C, info = P.posterior_cov(h, hyp, [xq], tol=tol, maxiter=maxiter)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        rec = {"n": 59_300, "m": m, "nq": nq, "tol": tol, "s": t,
               "iterations_max": info["iterations"], "converged": info["converged"],
               "min_diag": float(C.diagonal().min())}
        log(f"posterior covariance {nq}x{nq}, m={m}: {t*1e3:.1f} ms, "
            f"{info['iterations']} iterations")
        # rank-k covariance (k = min(m, 10000), Sec. 5): build once, then query
        k = min(m, 10000)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cache = P.love_build(h, hyp, k)
        torch.cuda.synchronize()
        t_build = time.perf_counter() - t0
        t0 = time.perf_counter()
        C_k = cache.cov([xq])
        torch.cuda.synchronize()
        t_query = time.perf_counter() - t0
        rec.update({"lowrank_k": k, "lowrank_rank": cache.rank, "lowrank_build_s": t_build,
                    "lowrank_query_s": t_query,
                    "lowrank_rel_frobenius": float(torch.linalg.norm(C_k - C) /
                                                   torch.linalg.norm(C))})
        log(f"rank-k covariance m={m}: rank {cache.rank}, build {t_build*1e3:.1f} ms, "
            f"query {t_query*1e3:.2f} ms, rel. Frobenius diff {rec['lowrank_rel_frobenius']:.2e}")
        cache.close()
        del C_k
        out.append(rec)
        h.close()
        del wl, C
        torch.cuda.empty_cache()
    return out


def main():
    args = _parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU per process and this benchmark on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    import paper_2101_11751_amd as P
    from paper_2101_11751_amd import workloads

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    P.load_library()
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    log(f"generating radar3d workload n={args.n} on {torch.cuda.get_device_name(0)}")
    wl = workloads.radar3d(n=args.n, device=dev)
    torch.cuda.synchronize()
    grid, hyp = wl["grid"], wl["hypers"]
    n = args.n
    # plain copy of a known size (256 MiB): the reference for scaling the
    # FETCH_SIZE / WRITE_SIZE counters of a profiled run
    calib = torch.empty(64 << 20, device=dev, dtype=torch.float32)
    calib2 = torch.empty_like(calib)
    calib2.copy_(calib)
    torch.cuda.synchronize()
    del calib, calib2

    def step(ev=None):
        if ev is not None:
            ev[0].record()
        h = P.precompute(grid, wl["x"], wl["y"], stats_dtype=torch.float32)
        if ev is not None:
            ev[1].record()
        mu, info = P.solve(h, hyp, tol=args.tol, maxiter=args.maxiter)
        if ev is not None:
            ev[2].record()
        return h, mu, info

    for w in range(args.warmup):
        h, mu, info = step()
        log(f"warmup {w}: iterations={info['iterations']} converged={info['converged']} "
            f"rel_res={info['rel_residual']:.2e}")
        h.close()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    iters = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        h, mu, info = step(evs[k])
        iters.append(info["iterations"])
        if k < args.steps - 1:
            h.close()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    t_pre = sum(e[0].elapsed_time(e[1]) for e in evs) / args.steps / 1e3
    t_sol = sum(e[1].elapsed_time(e[2]) for e in evs) / args.steps / 1e3
    log(f"timed {args.steps} steps: {elapsed:.3f} s; precompute {t_pre*1e3:.2f} ms, "
        f"solve {t_sol*1e3:.2f} ms, iterations {iters}")

    # dominant kernel: the banded W^T W product, launched as the CG loop
    # launches it (FP32 entries, FP64 vectors, u^T r reduced in the same
    # launch), timed with HIP events on the library's stream
    M = h.m_total
    x = torch.randn(M, device=dev, dtype=torch.float64)
    xp = P.padded(h, x, torch.float64)
    u = torch.empty(1, M, device=dev, dtype=torch.float64)
    P.wtw_matvec_dot(h, xp, u, reps=3)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    P.wtw_matvec_dot(h, xp, u, reps=args.mvm_reps)
    e1.record()
    torch.cuda.synchronize()
    t_spmv = e0.elapsed_time(e1) / args.mvm_reps / 1e3
    # cold: 512 MiB written between launches (flushes the 256 MiB MALL and L2)
    flush = torch.empty(128 << 20, device=dev, dtype=torch.float32)
    cold = []
    for r in range(10):
        flush.fill_(float(r))
        c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        c0.record()
        P.wtw_matvec_dot(h, xp, u, reps=1)
        c1.record()
        torch.cuda.synchronize()
        cold.append(c0.elapsed_time(c1) / 1e3)
    del flush
    t_cold = sum(cold) / len(cold)
    # algorithmic bytes: the exact nonzero FP32 entries, FP64 x read and u
    # written; beside it the bytes of the nonzero 64-row blocks it reads
    alg_bytes = 4 * h.nnz_wtw_nonzero + 8 * 2 * M
    block_bytes = 4 * h.wtw_blocks_nonzero * h.wtw_block_entries + 8 * 2 * M
    log(f"W^T W: {h.nnz_wtw_nonzero} nonzero entries; {h.wtw_blocks_nonzero} of "
        f"{h.wtw_blocks} blocks nonzero")
    achieved = alg_bytes / t_spmv / 1e9
    log(f"spmv (in-loop form) avg {t_spmv*1e6:.1f} us hot, {t_cold*1e6:.1f} us cold; "
        f"{achieved:.0f} GB/s on exact nonzeros, {block_bytes / t_spmv / 1e9:.0f} GB/s on blocks")
    # precompute: algorithmic bytes = the points read (x, y: 16 B each) and
    # the statistics written once (W^T W FP32 exact nonzeros, W^T y)
    pre_bytes = n * 4 * (h.d + 1) + 4 * h.nnz_wtw_nonzero + 8 * M
    # accuracy of the timed solve: against an FP64-statistics solve to 1e-8
    h64 = P.precompute(grid, wl["x"], wl["y"], stats_dtype=torch.float64)
    mu64, info64 = P.solve(h64, hyp, tol=1e-8, maxiter=200000)
    mean_err = float(torch.linalg.norm(mu - mu64) / torch.linalg.norm(mu64))
    log(f"timed solve's mean vs FP64 statistics at tol 1e-8 ({info64['iterations']} "
        f"iterations): rel. err {mean_err:.2e}")
    h64.close()
    del mu64

    iters_mean = sum(iters) / len(iters)
    result = {
        "metric": "precompute Mpts/s; CG MVMs/s at m=300k; MLL+grad s/eval vs plain FP64",
        "value": n * args.steps / elapsed / 1e6,
        "unit": "Mpts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "radar3d: n=1e8 cylinder r<=1, 0<=z<0.3, areal density ~1/(r+0.05), "
                               "50 anisotropic blobs + N(0,0.1^2); grid 100x100x30 (m=300000); "
                               "SE l=(0.05,0.05,0.02) s=1 sigma=0.1; FP32 inputs and stored W^T W, "
                               "FP64 operator arithmetic, FP64 CG vectors and scalars",
                   "n": n, "m": M, "tol": args.tol, "step": "precompute + posterior-mean solve"},
        "precompute_mpts_per_s": n / t_pre / 1e6,
        "precompute_ms": t_pre * 1e3,
        "precompute_alg_bytes": pre_bytes,
        "precompute_hbm_frac": pre_bytes / t_pre / 1e9 / HBM_PEAK_GBS,
        "solve_ms": t_sol * 1e3,
        "cg_iterations": iters_mean,
        "cg_mvms_per_s": iters_mean / t_sol,
        "mean_rel_err_vs_f64_tight": mean_err,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": SPMV_TRAFFIC_BYTES,
                     "kernel": "spmv_tiled_kernel<float,double,3> (banded W^T W product with "
                               "the fused u^T r reduction, as in the CG loop)",
                     "alg_bytes_per_launch": alg_bytes, "nnz_exact": h.nnz_wtw_nonzero,
                     "avg_launch_us": t_spmv * 1e6,
                     "block_bytes_per_launch": block_bytes,
                     "frac_on_nonzero_blocks": block_bytes / t_spmv / 1e9 / HBM_PEAK_GBS,
                     "cold_avg_launch_us": t_cold * 1e6,
                     "cold_frac": alg_bytes / t_cold / 1e9 / HBM_PEAK_GBS},
    }
    if not args.no_mll:
        torch.cuda.empty_cache()
        mc = mll_compare(P, workloads, torch, dev, args.mll_reps, args.mll_tol, args.mll_maxiter)
        result["mll_grad_s_per_eval"] = mc["batched_f32_s_per_eval"]
        result["mll_grad"] = mc
    if not args.no_extra:
        del h, mu
        torch.cuda.empty_cache()
        result["precompute_host"] = precompute_host_leg(P, torch, wl, n)
        result["precompute_2d"] = precompute_extra(P, workloads, torch, dev)
    if not args.no_batch:
        torch.cuda.empty_cache()
        bc = batch_compare(P, workloads, torch, dev, args.batch_tol, args.batch_maxiter,
                           loop_cmp=not args.no_batch_loop)
        result["batch_mll_grad_s_per_eval"] = bc["batched_s_per_eval"]
        result["batch_mll_grad"] = bc
    if not args.no_sweep:
        torch.cuda.empty_cache()
        result["ski_sweep"] = ski_sweep(P, workloads, torch, dev)
    if not args.no_sweep:
        torch.cuda.empty_cache()
        result["radar_per_iteration"] = radar_iter_leg(P, workloads, torch, dev)
    if not args.no_cov:
        torch.cuda.empty_cache()
        result["posterior_cov"] = cov_leg(P, workloads, torch, dev)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cb = cpu_baseline(wl, n, iters_mean, args.cpu_seconds)
        result["cpu_baseline"] = cb
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
