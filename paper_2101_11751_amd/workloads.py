"""Seeded synthetic workloads shaped like the paper's experiments.

This module only draws random inputs (points, responses, grid geometry and
hyperparameters).  It holds none of the method's arithmetic (no interpolation
weights, no sufficient statistics, no solver), so both the HIP path and the
oracle can consume its arrays.

Generation uses torch with an explicit generator on the requested device, so
a workload drawn on the GPU is reproducible on the GPU and one drawn on the
CPU is reproducible on the CPU (the two streams differ).  Every consumer that
compares two implementations hands both the same arrays.

Workloads (all kernels: squared exponential inside a scale kernel):
  sine1d   n=10,000 x~U[0,1], y = sin 6 pi x + 0.5 sin 20 pi x + N(0, 0.1^2),
           m=1000 on origin -0.01, spacing 1.02/999; l=0.05, s=1, sigma=0.1;
           FP64 throughout (the paper's synthetic sine, Sec. 5).
  bumps2d  n=1e6 x~U[0,1]^2, y = sum of 20 Gaussian bumps + N(0, 0.05^2),
           m=128x128; l=0.03, s=1, sigma=0.05; FP32 inputs.
  radar3d  n=1e8 points in the cylinder r<=1, 0<=z<0.3 with areal density
           proportional to 1/(r+0.05) (sweep-shaped sampling, standing in for
           the national radar network of Sec. 5), y = sum of 50 anisotropic
           Gaussian blobs + N(0, 0.1^2); m=100x100x30 on [-1,1]^2 x [0,0.3];
           l=(0.05,0.05,0.02), s=1, sigma=0.1; FP32 inputs.
  prior2d  n=4e6 x~U[0,1]^2, y drawn from a grid-structured GP prior (Def. 3)
           with l=0.04, s=1.5, sigma=0.1 on a 256x256 grid: grid values by
           circulant-embedding sampling on 512^2 (negative eigenvalues clipped)
           and a bilinear basis (the generator deliberately does not use the
           cubic basis of the method); 16 Rademacher probes, probe seed 4.
  batch64  64 independent problems of uneven size: 32 1-D (seed 1000+i:
           m = round(exp U[ln 512, ln 8192]), n = round(exp U[ln 1e4, ln 2e6]),
           data as sine1d with sigma = 0.1) and 32 2-D (seed 1032+i: square
           m x m grid, m ~ U{32..128}, n = round(exp U[ln 5e4, ln 1e6]), data as
           bumps2d with sigma = 0.05); l ~ U[0.01, 0.1] per problem, s = 1;
           31 Rademacher probes with probe seed 5000+i (32 right-hand sides
           [y, z_1 .. z_31] per problem); FP32 inputs.  Sizes and
           hyperparameters are drawn on the CPU (identical on every device),
           the data on the requested device.
The grid rule for the last four is h = (hi - lo)/(m - 3), origin = lo - h.
"""
import math

import torch

WORKLOADS = ("sine1d", "bumps2d", "radar3d", "prior2d", "batch64")


def padded_grid(m, lo, hi):
    d = len(m)
    lo = list(lo) if hasattr(lo, "__len__") else [lo] * d
    hi = list(hi) if hasattr(hi, "__len__") else [hi] * d
    h = [(hi[k] - lo[k]) / (m[k] - 3) for k in range(d)]
    return {"d": d, "m": list(m), "origin": [lo[k] - h[k] for k in range(d)],
            "spacing": h}


def _gen(seed, device):
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    return g


def sine1d(n=10_000, seed=0, device="cpu"):
    g = _gen(seed, device)
    x = torch.rand(n, generator=g, device=device, dtype=torch.float64)
    eps = torch.randn(n, generator=g, device=device, dtype=torch.float64) * 0.1
    y = torch.sin(6 * math.pi * x) + 0.5 * torch.sin(20 * math.pi * x) + eps
    grid = {"d": 1, "m": [1000], "origin": [-0.01], "spacing": [1.02 / 999]}
    hyp = {"lengthscale": [0.05], "outputscale": 1.0, "noise": 0.1}
    return {"name": "sine1d", "x": [x], "y": y, "grid": grid, "hypers": hyp,
            "dtype": torch.float64, "tol": 1e-8}


def sine1d_grid(n, m, seed=0, device="cpu"):
    """The synthetic sine data on a padded grid of m nodes over [0, 1] (for
    per-iteration sweeps over n and m)."""
    wl = sine1d(n=n, seed=seed, device=device)
    wl["grid"] = padded_grid([m], 0.0, 1.0)
    wl["name"] = f"sine1d n={n} m={m}"
    return wl


def bumps2d(n=1_000_000, seed=1, device="cpu", m=(128, 128), nbumps=20):
    g = _gen(seed, device)
    f64 = torch.float64
    x = torch.rand(2, n, generator=g, device=device, dtype=f64)
    c = torch.rand(nbumps, 2, generator=g, device=device, dtype=f64)
    w = 0.02 + 0.18 * torch.rand(nbumps, generator=g, device=device, dtype=f64)
    a = torch.randn(nbumps, generator=g, device=device, dtype=f64)
    eps = torch.randn(n, generator=g, device=device, dtype=f64) * 0.05
    y = eps.clone()
    for b in range(nbumps):
        r2 = (x[0] - c[b, 0]) ** 2 + (x[1] - c[b, 1]) ** 2
        y += a[b] * torch.exp(-r2 / (2 * w[b] ** 2))
    grid = padded_grid(list(m), 0.0, 1.0)
    hyp = {"lengthscale": [0.03, 0.03], "outputscale": 1.0, "noise": 0.05}
    return {"name": "bumps2d", "x": [x[0].float(), x[1].float()], "y": y.float(),
            "grid": grid, "hypers": hyp, "dtype": torch.float32, "tol": 1e-6}


def _radial_inverse_cdf(uu, a=0.05):
    """Inverse of F(r) = (r - a ln(1 + r/a)) / F(1) on [0,1] by bisection
    (areal density proportional to 1/(r+a) means p(r) ~ r/(r+a))."""
    F1 = 1.0 - a * math.log(1.0 + 1.0 / a)
    target = uu * F1
    lo = torch.zeros_like(uu)
    hi = torch.ones_like(uu)
    for _ in range(40):
        mid = 0.5 * (lo + hi)
        f = mid - a * torch.log1p(mid / a)
        below = f < target
        lo = torch.where(below, mid, lo)
        hi = torch.where(below, hi, mid)
    return 0.5 * (lo + hi)


def radar3d(n=100_000_000, seed=2, device="cpu", m=(100, 100, 30), nblobs=50,
            chunk=1 << 24):
    """Cylinder of radius 1 and height 0.3, sweep-shaped radial density."""
    g = _gen(seed, device)
    f32 = torch.float32
    f64 = torch.float64
    # blob parameters first (drawn in a fixed order), then the points in chunks
    br = _radial_inverse_cdf(torch.rand(nblobs, generator=g, device=device, dtype=f64))
    bphi = 2 * math.pi * torch.rand(nblobs, generator=g, device=device, dtype=f64)
    bz = 0.3 * torch.rand(nblobs, generator=g, device=device, dtype=f64)
    bc = torch.stack([br * torch.cos(bphi), br * torch.sin(bphi), bz], 1)
    wxy = 0.05 + 0.25 * torch.rand(nblobs, 2, generator=g, device=device, dtype=f64)
    wz = 0.02 + 0.08 * torch.rand(nblobs, 1, generator=g, device=device, dtype=f64)
    bw = torch.cat([wxy, wz], 1)
    amp = torch.randn(nblobs, generator=g, device=device, dtype=f64)
    X = torch.empty(3, n, device=device, dtype=f32)
    Y = torch.empty(n, device=device, dtype=f32)
    for s0 in range(0, n, chunk):
        k = min(chunk, n - s0)
        r = _radial_inverse_cdf(torch.rand(k, generator=g, device=device, dtype=f32)).clamp_(0, 1)
        phi = (2 * math.pi) * torch.rand(k, generator=g, device=device, dtype=f32)
        z = 0.3 * torch.rand(k, generator=g, device=device, dtype=f32)
        px = (r * torch.cos(phi)).clamp_(-1, 1)
        py = (r * torch.sin(phi)).clamp_(-1, 1)
        yy = 0.1 * torch.randn(k, generator=g, device=device, dtype=f32)
        for b in range(nblobs):
            q = (((px - bc[b, 0]) / bw[b, 0]) ** 2 + ((py - bc[b, 1]) / bw[b, 1]) ** 2
                 + ((z - bc[b, 2]) / bw[b, 2]) ** 2)
            yy += amp[b].float() * torch.exp(-0.5 * q.float())
        X[0, s0:s0 + k] = px
        X[1, s0:s0 + k] = py
        X[2, s0:s0 + k] = z
        Y[s0:s0 + k] = yy
    grid = padded_grid(list(m), [-1.0, -1.0, 0.0], [1.0, 1.0, 0.3])
    hyp = {"lengthscale": [0.05, 0.05, 0.02], "outputscale": 1.0, "noise": 0.1}
    return {"name": "radar3d", "x": [X[0], X[1], X[2]], "y": Y, "grid": grid,
            "hypers": hyp, "dtype": f32, "tol": 1e-6}


def _grid_prior_sample(g, device, m, h, ell, s, L):
    """theta ~ N(0, K_G) for a separable SE kernel on an m[0] x m[1] grid by
    circulant embedding on L x L (negative spectrum clipped to 0).  Returns
    (theta [m0, m1] float64, clipped fraction of the spectrum mass)."""
    f64 = torch.float64
    lam = None
    for k in range(2):
        j = torch.arange(L, device=device, dtype=f64)
        dist = torch.minimum(j, L - j) * h[k]
        col = torch.exp(-0.5 * (dist / ell) ** 2)
        lk = torch.fft.fft(col).real
        lam = lk if lam is None else lam[:, None] * lk[None, :]
    lam = s * lam
    neg = float(lam.clamp(max=0).abs().sum() / lam.abs().sum())
    lam = lam.clamp(min=0)
    e = torch.complex(torch.randn(L, L, generator=g, device=device, dtype=f64),
                      torch.randn(L, L, generator=g, device=device, dtype=f64))
    f = torch.fft.fft2(torch.sqrt(lam / (L * L)) * e)
    theta = f.real[:m[0], :m[1]]
    return theta, neg


def prior2d(n=4_000_000, seed=3, device="cpu", m=(256, 256), probe_seed=4, nprobes=16):
    g = _gen(seed, device)
    f64 = torch.float64
    grid = padded_grid(list(m), 0.0, 1.0)
    true = {"lengthscale": [0.04, 0.04], "outputscale": 1.5, "noise": 0.1}
    L = 2 * max(m)
    theta, clipped = _grid_prior_sample(g, device, m, grid["spacing"], 0.04, 1.5, L)
    x = torch.rand(2, n, generator=g, device=device, dtype=f64)
    # bilinear basis on the same grid
    u0 = (x[0] - grid["origin"][0]) / grid["spacing"][0]
    u1 = (x[1] - grid["origin"][1]) / grid["spacing"][1]
    i0 = torch.clamp(torch.floor(u0).long(), 0, m[0] - 2)
    i1 = torch.clamp(torch.floor(u1).long(), 0, m[1] - 2)
    t0 = u0 - i0
    t1 = u1 - i1
    f = ((1 - t0) * (1 - t1) * theta[i0, i1] + t0 * (1 - t1) * theta[i0 + 1, i1]
         + (1 - t0) * t1 * theta[i0, i1 + 1] + t0 * t1 * theta[i0 + 1, i1 + 1])
    y = f + 0.1 * torch.randn(n, generator=g, device=device, dtype=f64)
    offset = {"lengthscale": [0.05, 0.05], "outputscale": 1.0, "noise": 0.15}
    return {"name": "prior2d", "x": [x[0].float(), x[1].float()], "y": y.float(),
            "grid": grid, "hypers": true, "hypers_offset": offset,
            "dtype": torch.float32, "probe_seed": probe_seed, "nprobes": nprobes,
            "lanczos_steps": 30, "clipped_spectrum_fraction": clipped, "tol": 1e-6}


def _batch_problem(i, device, n_scale, nprobes):
    """Problem i of batch64 (0 <= i < 32: 1-D, 32 <= i < 64: 2-D)."""
    seed = 1000 + i
    gc = _gen(seed, "cpu")
    f64 = torch.float64
    u = torch.rand(3, generator=gc, dtype=f64)
    if i < 32:
        m = [int(round(math.exp(math.log(512) + u[0].item() * math.log(8192 / 512))))]
        n = int(round(math.exp(math.log(1e4) + u[1].item() * math.log(2e6 / 1e4))))
        sigma = 0.1
    else:
        md = 32 + int(torch.randint(0, 97, (1,), generator=gc).item())
        m = [md, md]
        n = int(round(math.exp(math.log(5e4) + u[1].item() * math.log(1e6 / 5e4))))
        sigma = 0.05
    ell = 0.01 + 0.09 * u[2].item()
    n = max(16, int(round(n * n_scale)))
    g = _gen(seed, device)
    d = len(m)
    x = torch.rand(d, n, generator=g, device=device, dtype=f64)
    if d == 1:
        y = (torch.sin(6 * math.pi * x[0]) + 0.5 * torch.sin(20 * math.pi * x[0])
             + sigma * torch.randn(n, generator=g, device=device, dtype=f64))
    else:
        nb = 20
        c = torch.rand(nb, 2, generator=g, device=device, dtype=f64)
        w = 0.02 + 0.18 * torch.rand(nb, generator=g, device=device, dtype=f64)
        a = torch.randn(nb, generator=g, device=device, dtype=f64)
        y = sigma * torch.randn(n, generator=g, device=device, dtype=f64)
        for b in range(nb):
            r2 = (x[0] - c[b, 0]) ** 2 + (x[1] - c[b, 1]) ** 2
            y += a[b] * torch.exp(-r2 / (2 * w[b] ** 2))
    return {"name": f"batch64[{i}]", "x": [x[k].float() for k in range(d)], "y": y.float(),
            "grid": padded_grid(m, 0.0, 1.0),
            "hypers": {"lengthscale": [ell] * d, "outputscale": 1.0, "noise": sigma},
            "dtype": torch.float32, "probe_seed": 5000 + i, "nprobes": nprobes,
            "lanczos_steps": 30, "n": n, "m": m}


def batch64(device="cpu", n_scale=1.0, nprobes=31, which=None):
    """List of the batch64 problems (all 64, or the indices in `which`);
    n_scale shrinks every n (for tests)."""
    idx = range(64) if which is None else which
    return [_batch_problem(i, device, n_scale, nprobes) for i in idx]


def get(name, **kw):
    return {"sine1d": sine1d, "bumps2d": bumps2d, "radar3d": radar3d,
            "prior2d": prior2d, "batch64": batch64}[name](**kw)
