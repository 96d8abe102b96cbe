"""Writes the FP64 oracle's posterior mean for the 2-D bumps workload
(n = 10^6 on [0,1]^2, 128 x 128 grid, l = 0.03, s = 1, sigma = 0.05) to
bumps2d_reference.npz, with the SHA-256 of the input arrays it was computed
from.  Only the oracle computes the stored values (its factorized CG solved
to a relative residual of 1e-13: about 18,000 iterations, too slow to run
inside a GPU test).

    python tests/golden/make_bumps2d_reference.py
"""
import hashlib
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2101_11751_amd import workloads  # noqa: E402

OUT = os.path.join(HERE, "bumps2d_reference.npz")


def inputs():
    """The workload's arrays as the tests use them (drawn on the CPU)."""
    wl = workloads.bumps2d()
    X = np.stack([x.numpy() for x in wl["x"]])          # float32 [2, n]
    y = wl["y"].numpy()                                 # float32 [n]
    return wl, X, y


def digest(X, y):
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(X).tobytes())
    h.update(np.ascontiguousarray(y).tobytes())
    return h.hexdigest()


def main():
    wl, X, y = inputs()
    wtw, wty, yty = oracle.precompute(wl["grid"], X, y)
    mu, _, info = oracle.solve_mean(wl["grid"], wl["hypers"], wtw, wty, yty, tol=1e-13,
                                    maxiter=100000)
    np.savez(OUT, mu_G=mu, iterations=info["iterations"], sha256=digest(X, y), tol=1e-13)
    print(f"wrote {OUT}: {info['iterations']} iterations")


if __name__ == "__main__":
    main()
