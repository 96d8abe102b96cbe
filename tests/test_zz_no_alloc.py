"""fkgp_solve_noalloc (the solve for callers that cannot allocate) against
fkgp_solve, through the C ABI: two calls in a row, the second on a smaller
grid (the fixed workspace keeps the first call's contents), each equal to
fkgp_solve bit for bit; no device allocation through the library's
allocator during either call; grids too large for the workspace are refused
before any launch."""
import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2101_11751_amd")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def handle(seed, m, n, stats):
    rng = np.random.default_rng(seed)
    d = len(m)
    grid = oracle.make_grid(m, lo=0.0, hi=1.0)
    X = rng.uniform(0, 1, (d, n)).astype(np.float32)
    y = (np.sin(5 * X[0].astype(np.float64)) + 0.2 * rng.standard_normal(n)).astype(np.float32)
    xs = [torch.from_numpy(np.ascontiguousarray(X[k])).cuda() for k in range(d)]
    return P.precompute(grid, xs, torch.from_numpy(y).cuda(), stats_dtype=stats)


HYP = {2: {"lengthscale": [0.06, 0.07], "outputscale": 1.2, "noise": 0.2},
       3: {"lengthscale": [0.1, 0.12, 0.15], "outputscale": 0.9, "noise": 0.25}}


def counting_allocator():
    alloc_t, free_t = P.torch_allocator()
    calls = {"alloc": 0, "free": 0}

    def alloc(n, stream):
        calls["alloc"] += 1
        return alloc_t(n, stream)

    def free(ptr, stream):
        calls["free"] += 1
        free_t(ptr, stream)

    return alloc, free, calls


@pytest.mark.parametrize("stats,op", [(torch.float32, "f64"), (torch.float32, "stats"),
                                      (torch.float64, "f64")])
def test_noalloc_solve_equals_solve_twice_then_smaller(stats, op):
    _need_gpu()
    big = handle(1, [60, 50, 40], 200000, stats)      # 120,000 nodes
    small = handle(2, [37, 29], 30000, stats)         # 1,073 nodes
    cases = [(big, HYP[3], None), (small, HYP[2], None),
             (small, HYP[2], torch.from_numpy(np.random.default_rng(3).standard_normal(
                 small.m_total)).cuda())]
    refs = [P.solve(h, hp, rhs=r, tol=1e-9, maxiter=5000, op_precision=op)
            for h, hp, r in cases]
    outs = [torch.full((h.m_total,), float("nan"), dtype=torch.float64, device="cuda")
            for h, _, _ in cases]
    torch.cuda.synchronize()
    alloc, free, calls = counting_allocator()
    P.set_allocator(alloc, free)
    try:
        infos = [P.solve(h, hp, rhs=r, tol=1e-9, maxiter=5000, op_precision=op, out=o,
                         noalloc=True)[1]
                 for (h, hp, r), o in zip(cases, outs)]
    finally:
        P.set_allocator()
    assert calls["alloc"] == 0 and calls["free"] == 0
    for (ref, rinfo), out, info in zip(refs, outs, infos):
        assert info["converged"] and info["iterations"] == rinfo["iterations"]
        assert info["rel_residual"] == rinfo["rel_residual"]
        assert torch.equal(out, ref)


def test_noalloc_refuses_grids_beyond_its_workspace():
    _need_gpu()
    h = handle(4, [120, 110, 100], 20000, torch.float32)   # 1.32M nodes: ~110 MB of workspace
    out = torch.empty(h.m_total, dtype=torch.float64, device="cuda")
    with pytest.raises(P.FkgpError, match="workspace"):
        P.solve(h, HYP[3], tol=1e-6, maxiter=10, out=out, noalloc=True)
    # the refusal launched nothing: a solve afterwards is unaffected
    small = handle(5, [20, 24], 5000, torch.float32)
    a, _ = P.solve(small, HYP[2], tol=1e-9, maxiter=3000, noalloc=True)
    b, _ = P.solve(small, HYP[2], tol=1e-9, maxiter=3000)
    assert torch.equal(a, b)
