"""Write oracle reference samples of the full-size Taylor-Green runs.

The large parity cases (the 256^3 TGV after 100 RK3 steps, the 512^3 TGV
after 50) take the FP64 oracle tens of minutes to hours, too long to run
inside a test.  This script runs them once with the oracle alone and stores
what a GPU test needs to compare a state element by element at sampled
points:

  points     linear point indices (random points incl. the 8 corners, plus
             one full x-, y- and z-line through a random point, so every tile
             and z-chunk boundary along those lines is crossed)
  values     the oracle state at those points, shape (npoints, 5)
  field_max  max |x| of each field over the whole grid (the scale of the
             per-field relative error)
  sum, sumsq per-field sums of x and x^2 over the whole grid
  diag       the oracle's eight diagnostics of the final state

Only ``oracle`` and ``synth`` (parameters, time step, sample points) are
used; nothing here comes from the GPU path.

Usage:  python tests/golden/make_tgv_oracle_samples.py N STEPS
        (OMP_NUM_THREADS sets the oracle's threads)
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

SAMPLE_SEED = 20170927
RANDOM_POINTS = 1024


def sample_indices(n: int) -> np.ndarray:
    shape = (n, n, n)
    pts = set(synth.sample_points(shape, RANDOM_POINTS, SAMPLE_SEED).tolist())
    rng = np.random.default_rng(SAMPLE_SEED + 1)
    i0, j0, k0 = (int(v) for v in rng.integers(0, n, size=3))
    for t in range(n):
        pts.add((k0 * n + j0) * n + t)      # x-line
        pts.add((k0 * n + t) * n + i0)      # y-line
        pts.add((t * n + j0) * n + i0)      # z-line
    return np.array(sorted(pts), dtype=np.int64)


def golden_path(n: int, steps: int) -> str:
    return os.path.join(HERE, f"tgv{n}_{steps}steps_oracle.npz")


def main(n: int, steps: int) -> str:
    ph = oracle.Physics(n=(n, n, n))
    dt = synth.stable_dt(n, ph.mach)
    t0 = time.perf_counter()
    Q = oracle.rk3(ph, oracle.tgv_init(ph), dt, steps)
    sec = time.perf_counter() - t0
    pts = sample_indices(n)
    flat = Q.reshape(5, -1)
    values = np.ascontiguousarray(flat[:, pts].T)
    field_max = np.abs(flat).max(axis=1)
    s = flat.sum(axis=1)
    s2 = np.einsum("ij,ij->i", flat, flat)
    d = oracle.diagnostics(ph, Q)
    diag = np.array([d[k] for k in oracle.DIAG_NAMES])
    out = golden_path(n, steps)
    np.savez(out, n=n, steps=steps, dt=dt, gamma=ph.gamma, prandtl=ph.prandtl,
             reynolds=ph.reynolds, mach=ph.mach, points=pts, values=values,
             field_max=field_max, sum=s, sumsq=s2, diag=diag,
             oracle_seconds=sec, oracle_threads=int(os.environ.get("OMP_NUM_THREADS", "0")))
    print(f"{out}: {pts.size} points, oracle {sec:.0f} s", flush=True)
    return out


if __name__ == "__main__":
    main(int(sys.argv[1]), int(sys.argv[2]))
