"""Seeded synthetic inputs shared by the tests, the benchmark and the
oracle checks.

This module holds no arithmetic of the method (no equation of state, no
stencil, no residual, no time integration): it only draws random numbers and
lays them out as conserved-variable arrays, instance tables and request
streams.  Both the HIP path and the oracle consume what it produces.

Workload recipe (arXiv:1709.09713, results section): the paper runs one
Taylor-Green vortex at 256^3 with Re = 1600, Pr = 0.71, M = 0.1,
gamma = 1.4.  That initial state is analytic, so each side computes it itself
(``tgv_init``); what is drawn here are (a) perturbed conserved states used to
exercise every stencil tap, (b) the per-instance parameters of batched runs
(grid size, Reynolds and Mach numbers) and (c) Poisson request streams.
"""
from __future__ import annotations

import numpy as np

PAPER_GAMMA = 1.4
PAPER_PRANDTL = 0.71
PAPER_REYNOLDS = 1600.0
PAPER_MACH = 0.1


def stable_dt(n: int, mach: float) -> float:
    """Time step for an n^3 grid.  The paper prints no dt; 3.385e-3 is the
    16^3 step, and for finer grids or faster sound it is scaled with the
    grid spacing and with (1 + M)/M so that the explicit RK3 stability
    number stays below about 0.9 (a fixed 3.385e-3 diverges from 128^3 up)."""
    return min(3.385e-3, 3.385e-3 * (64.0 / n) * 11.0 * mach / (1.0 + mach))


def _smooth_modes(rng, shape, nmodes, amp):
    """Sum of ``nmodes`` random low-wavenumber Fourier modes on the periodic
    grid of ``shape`` = (nz, ny, nx), scaled to max amplitude ~amp."""
    nz, ny, nx = shape
    z = np.arange(nz)[:, None, None] * (2 * np.pi / nz)
    y = np.arange(ny)[None, :, None] * (2 * np.pi / ny)
    x = np.arange(nx)[None, None, :] * (2 * np.pi / nx)
    f = np.zeros(shape)
    for _ in range(nmodes):
        kx, ky, kz = rng.integers(-3, 4, size=3)
        ph = rng.uniform(0, 2 * np.pi)
        a = rng.uniform(-1, 1)
        f += a * np.cos(kx * x + ky * y + kz * z + ph)
    return amp * f / max(1.0, nmodes ** 0.5)


def random_state(shape, seed: int, *, energy_mean: float = 180.0,
                 noise: float = 0.05, smooth: float = 0.5):
    """Conserved state Q[5, nz, ny, nx] = (rho, m0, m1, m2, rhoE) with
    rho ~ 1, |m| ~ smooth, rhoE ~ energy_mean, plus white noise of relative
    size ``noise`` so every stencil tap matters.  energy_mean = 180 is the
    order of rhoE at M = 0.1 (pressure stays positive for these amplitudes).
    """
    rng = np.random.default_rng(seed)
    shape = tuple(shape)
    Q = np.empty((5,) + shape)
    Q[0] = 1.0 + _smooth_modes(rng, shape, 6, 0.1 * smooth) \
        + 0.1 * noise * rng.uniform(-1, 1, shape)
    for v in (1, 2, 3):
        Q[v] = _smooth_modes(rng, shape, 6, smooth) \
            + noise * rng.uniform(-1, 1, shape)
    Q[4] = energy_mean + _smooth_modes(rng, shape, 6, smooth) \
        + noise * rng.uniform(-1, 1, shape)
    return Q


def resting_density_mode(shape, direction: int, mode: int, eps: float,
                         energy: float):
    """Conserved state Q[5, nz, ny, nx] of a fluid at rest with a density
    wave along one direction: rho = 1 / (1 + eps cos(theta)),
    theta = 2 pi mode i_d / n_d, zero momentum and uniform rho E = energy.
    (The fluid is at rest and, for a uniform rho E, at uniform pressure, so
    only heat conduction acts on it.)"""
    nz, ny, nx = shape
    n_d = (nx, ny, nz)[direction]
    idx = np.arange(n_d) * (2 * np.pi * mode / n_d)
    bshape = [1, 1, 1]
    bshape[2 - direction] = n_d
    theta = np.broadcast_to(idx.reshape(bshape), shape)
    Q = np.zeros((5,) + tuple(shape))
    Q[0] = 1.0 / (1.0 + eps * np.cos(theta))
    Q[4] = energy
    return Q


def sample_points(shape, count: int, seed: int):
    """``count`` distinct linear point indices of a grid of ``shape``
    (nz, ny, nx), always including the eight corners (wrap-around cases)."""
    nz, ny, nx = shape
    total = nx * ny * nz
    rng = np.random.default_rng(seed)
    corners = [((k * ny) + j) * nx + i for k in (0, nz - 1) for j in (0, ny - 1)
               for i in (0, nx - 1)]
    pts = set(corners)
    want = min(count, total)
    while len(pts) < want:
        pts.update(rng.integers(0, total, size=want - len(pts)).tolist())
    return np.array(sorted(pts), dtype=np.int64)


BATCH_SIZES = (32, 48, 64, 96, 128)
SERVE_SIZES = (32, 48, 64, 96, 128, 160, 192)


def batch_instances(seed: int, count: int = 64, sizes=BATCH_SIZES,
                    steps: int = 200):
    """Independent TGV instances for batched runs: N uniform over ``sizes``,
    Re ~ U[400, 3200], M ~ U[0.05, 0.4], dt from ``stable_dt``."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.choice(sizes))
        re = float(rng.uniform(400.0, 3200.0))
        mach = float(rng.uniform(0.05, 0.4))
        out.append(dict(n=n, reynolds=re, mach=mach, dt=stable_dt(n, mach),
                        steps=steps))
    return out


def poisson_requests(seed: int, count: int, rate_hz: float = 50.0,
                     sizes=SERVE_SIZES, steps_range=(100, 1000)):
    """A Poisson arrival stream: exponential gaps of mean 1/rate_hz seconds;
    each request draws N from ``sizes``, Re ~ U[400, 3200],
    M ~ U[0.05, 0.4] and a step count uniform in ``steps_range``."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for rid in range(count):
        t += float(rng.exponential(1.0 / rate_hz))
        n = int(rng.choice(sizes))
        re = float(rng.uniform(400.0, 3200.0))
        mach = float(rng.uniform(0.05, 0.4))
        steps = int(rng.integers(steps_range[0], steps_range[1] + 1))
        out.append(dict(rid=rid, arrival=t, n=n, reynolds=re, mach=mach,
                        dt=stable_dt(n, mach), steps=steps))
    return out
