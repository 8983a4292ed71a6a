"""Pins of the oracle's residual, Runge-Kutta update and diagnostics against
what the paper and the mathematics fix (CPU only).

Each test names the property and why a plausible slip in the oracle (a
dropped term, a wrong sign or index, a transposed operand) would fail it.
"""
import math

import numpy as np
import pytest

import synth
from closed_forms import HEAT_CASES, heat_mode_expected
from oracle import numpy_ref

INF = float("inf")


def sigma1(m, h):
    return (8 * math.sin(m * h) - math.sin(2 * m * h)) / (6 * h)


def sigma2(m, h):
    return (2.5 - (8 / 3) * math.cos(m * h) + math.cos(2 * m * h) / 6) / h ** 2


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


SHAPES = [(12, 10, 14), (5, 6, 7), (16, 16, 16), (9, 13, 5)]


@pytest.mark.parametrize("n", SHAPES)
@pytest.mark.parametrize("re", [1600.0, 400.0, INF])
def test_c_oracle_matches_independent_numpy(orc, n, re):
    """Two implementations of the methodology-section equations written in
    different arithmetic forms (eq. (fd) coefficients vs the listing's
    8(f+1 - f-1) form; literal viscous bracket vs hand-simplified one)."""
    ph = orc.Physics(n=n, reynolds=re, mach=0.2)
    Q = synth.random_state(n[::-1], seed=sum(n))
    R = orc.residual(ph, Q)
    Rn = numpy_ref.residual(Q, ph.h, ph.gamma, ph.prandtl, ph.reynolds, ph.mach)
    for v in range(5):
        assert _rel(R[v], Rn[v]) < 2e-13, v


def test_uniform_state_has_zero_residual(orc):
    """A uniform state is an exact steady solution."""
    ph = orc.Physics(n=(8, 7, 6))
    Q = np.empty((5, 6, 7, 8))
    Q[0], Q[1], Q[2], Q[3], Q[4] = 1.3, 0.4, -0.2, 0.7, 200.0
    R = orc.residual(ph, Q)
    assert np.abs(R).max() < 1e-12


@pytest.mark.parametrize("case", [0, 1])
@pytest.mark.parametrize("d", [0, 1, 2])
@pytest.mark.parametrize("m", [1, 2])
def test_heat_conduction_closed_form(orc, case, d, m):
    """A resting fluid at uniform pressure with a temperature wave along
    x_d: mass and momentum residuals are exactly zero and the energy
    residual is the heat-conduction term alone, in closed form (see
    heat_mode_expected).  Pins kappa (every factor: gamma - 1, M^2, Pr, Re),
    T from eq. (Tinprimitive), the direction of each D2_j T and the sign."""
    n, length, g, pr, re, mach = HEAT_CASES[case]
    eps = 0.05
    energy = 1.0 / (g * (g - 1.0) * mach ** 2)      # p = 1 / (gamma M^2)
    ph = orc.Physics(n=n, length=length, gamma=g, prandtl=pr, reynolds=re, mach=mach)
    Q = synth.resting_density_mode(n[::-1], d, m, eps, energy)
    R = orc.residual(ph, Q)
    assert np.all(R[:4] == 0.0)
    want = heat_mode_expected(HEAT_CASES[case], d, m, eps, energy)
    assert _rel(R[4], want) < 1e-12


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_discrete_conservation(orc, seed):
    """Skew-symmetric convection with an antisymmetric periodic D conserves
    mass, momentum and (inviscid) energy to rounding; with viscosity the
    energy sum equals the closed-form leak of the Laplacian-form split."""
    n = (10, 12, 8)
    Q = synth.random_state(n[::-1], seed=seed)
    for re in (INF, 800.0):
        ph = orc.Physics(n=n, reynolds=re, mach=0.15)
        R = orc.residual(ph, Q)
        for v in range(4):
            assert abs(R[v].sum()) < 1e-13 * np.abs(R[v]).sum(), (re, v)
        if math.isinf(re):
            assert abs(R[4].sum()) < 1e-13 * np.abs(R[4]).sum()
        else:
            leak = numpy_ref.energy_leak(Q, ph.h, re)
            assert abs(leak) > 1e-6 * np.abs(R[4]).sum()  # a real, nonzero leak
            assert abs(R[4].sum() - leak) < 1e-13 * np.abs(R[4]).sum()


def test_energy_leak_is_fourth_order_small(orc):
    """The viscous energy leak is a truncation error: it must shrink like
    h^4 on a smooth field under refinement, not grow."""
    leaks = []
    for n in (16, 32):
        ph = orc.Physics(n=(n, n, n))
        Q = orc.tgv_init(ph)
        R = orc.residual(ph, Q)
        leaks.append(abs(R[4].sum()) / n ** 3)
    assert leaks[1] < leaks[0] / 10


def test_axis_permutation_symmetry(orc):
    """Swapping x and y (and u and v) permutes the residual."""
    n = (9, 9, 7)
    ph = orc.Physics(n=n, mach=0.2)
    Q = synth.random_state(n[::-1], seed=5)
    Qs = Q[[0, 2, 1, 3, 4]].transpose(0, 1, 3, 2).copy()
    R = orc.residual(ph, Q)
    Rs = orc.residual(ph, Qs)
    Rback = Rs[[0, 2, 1, 3, 4]].transpose(0, 1, 3, 2)
    for v in range(5):
        assert _rel(Rback[v], R[v]) < 1e-14


def test_one_dimensional_state_stays_one_dimensional(orc):
    """A state that varies only along x with v = w = 0 has R_m1 = R_m2 = 0
    exactly: fd stencils are exact differences, so no y or z derivative
    leaks in.  Catches a direction or component index mix-up."""
    n = (16, 5, 6)
    ph = orc.Physics(n=n, mach=0.3)
    Q1 = synth.random_state((1, 1, 16), seed=7)
    Q = np.broadcast_to(Q1, (5, 6, 5, 16)).copy()
    Q[2] = 0.0
    Q[3] = 0.0
    R = orc.residual(ph, Q)
    assert np.all(R[2] == 0.0) and np.all(R[3] == 0.0)
    assert np.abs(R[1]).max() > 1e-3
    # and the x-dependence is the same on every (y, z) line
    assert np.all(R[0] == R[0][:1, :1, :])


def test_residual_self_convergence(orc):
    """R(Q0) of the TGV on nested grids converges at fourth order."""
    Rs = {}
    for n in (16, 32, 64):
        ph = orc.Physics(n=(n, n, n))
        Rs[n] = orc.residual(ph, orc.tgv_init(ph))
    d1 = np.abs(Rs[16] - Rs[32][:, ::2, ::2, ::2]).max(axis=(1, 2, 3))
    d2 = np.abs(Rs[32] - Rs[64][:, ::2, ::2, ::2]).max(axis=(1, 2, 3))
    for v in range(5):
        if d2[v] > 1e-13:
            ratio = d1[v] / d2[v]
            assert 12.0 < ratio < 20.0, (v, ratio)


@pytest.mark.parametrize("n", [8, 16, 32])
def test_tgv_initial_diagnostics_closed_forms(orc, n):
    """t = 0 diagnostics of the results-section initial state: mean rho = 1,
    KE = 1/8, mean rhoE = 1/(gamma(gamma-1)M^2) + 1/8, zero momentum and
    rho-weighted enstrophy sigma1(1)^2 (3/8 - 5 gamma M^2 / 128)."""
    g, M, re = 1.4, 0.1, 1600.0
    ph = orc.Physics(n=(n, n, n), gamma=g, mach=M, reynolds=re)
    d = orc.diagnostics(ph, orc.tgv_init(ph))
    vol = (2 * math.pi) ** 3
    assert d["mass"] == pytest.approx(vol, rel=1e-12)
    assert d["energy"] == pytest.approx(vol * (1 / (g * (g - 1) * M * M) + 0.125), rel=1e-12)
    assert d["kinetic_energy"] == pytest.approx(0.125, rel=1e-13)
    for c in ("momentum_x", "momentum_y", "momentum_z"):
        assert abs(d[c]) < 1e-12
    s1 = sigma1(1, 2 * math.pi / n)
    omega = s1 ** 2 * (3 / 8 - 5 * g * M * M / 128)
    assert d["enstrophy"] == pytest.approx(omega, rel=1e-13)
    assert d["dissipation"] == pytest.approx(2 * omega / re, rel=1e-13)


def test_tgv_init_fields(orc):
    """The initial velocity and pressure of the results section, recovered
    from the conserved variables, and T = 1."""
    n = 12
    g, M = 1.4, 0.1
    ph = orc.Physics(n=(n, n, n))
    Q = orc.tgv_init(ph)
    x = np.arange(n) * 2 * math.pi / n
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    u = Q[1] / Q[0]
    v = Q[2] / Q[0]
    np.testing.assert_allclose(u, np.sin(X) * np.cos(Y) * np.cos(Z), atol=1e-14)
    np.testing.assert_allclose(v, -np.cos(X) * np.sin(Y) * np.cos(Z), atol=1e-14)
    assert np.all(Q[3] == 0.0)
    p = 1 / (g * M * M) + (np.cos(2 * X) + np.cos(2 * Y)) * (2 + np.cos(2 * Z)) / 16
    np.testing.assert_allclose(Q[0], g * M * M * p, rtol=1e-14)


def test_rk3_conserves_sums(orc):
    """The RK update is linear in R, so sum(Q) of mass and momentum is
    preserved to rounding over many steps."""
    n = (12, 12, 12)
    ph = orc.Physics(n=n)
    Q0 = orc.tgv_init(ph)
    Q = orc.rk3(ph, Q0, 3.385e-3, 5)
    for v in range(4):
        assert abs(Q[v].sum() - Q0[v].sum()) < 1e-12 * np.abs(Q0[v]).sum() + 1e-12


@pytest.mark.parametrize("mach,dt", [(0.1, 3.385e-3), (0.05, 1.6925e-3)])
def test_early_kinetic_energy_decay(orc, mach, dt):
    """At early times the TGV kinetic energy decays like the incompressible
    closed form (1/8) exp(-6 sigma2(1) t / Re): each velocity component has
    |k|^2 = 3 and the vortex stretching vanishes at t = 0.  A wrong viscous
    sign, factor or Reynolds scaling misses by O(1)."""
    n, steps, re = 32, 20, 1600.0
    ph = orc.Physics(n=(n, n, n), mach=mach, reynolds=re)
    Q0 = orc.tgv_init(ph)
    Q = orc.rk3(ph, Q0, dt, steps)
    ke0 = orc.diagnostics(ph, Q0)["kinetic_energy"]
    ke = orc.diagnostics(ph, Q)["kinetic_energy"]
    t = dt * steps
    closed = 0.125 * math.exp(-6 * sigma2(1, 2 * math.pi / n) * t / re) - 0.125
    assert abs((ke - ke0) / closed - 1) < 3e-3


def _acoustic_state(nx, eps, m, g, M):
    h = 2 * math.pi / nx
    x = np.arange(nx) * h
    c, p0 = 1 / M, 1 / (g * M * M)
    pp = eps * np.cos(m * x)
    u = pp / c
    rho = 1 + pp / c ** 2
    p = p0 + pp
    Q = np.empty((5, 5, 5, nx))
    Q[0], Q[1], Q[2], Q[3] = rho, rho * u, 0.0, 0.0
    Q[4] = p / (g - 1) + 0.5 * rho * u * u
    return Q


@pytest.mark.parametrize("m", [1, 3, 6])
def test_linear_acoustics_amplification(orc, m):
    """An inviscid small-amplitude right-running acoustic wave: per RK3 step
    its complex amplitude is multiplied by P(z) = 1 + z + z^2/2 + z^3/6 with
    z = -i c sigma1(m) dt, c = 1/M.  Pins the equation of state, the skew
    convection, the pressure work and the RK3 polynomial together; the
    +eps/-eps difference cancels O(eps^2)."""
    g, M, nx, steps, eps = 1.4, 0.1, 32, 10, 1e-4
    ph = orc.Physics(n=(nx, 5, 5), reynolds=INF, gamma=g, mach=M)
    h = 2 * math.pi / nx
    dt = 0.2 * h * M

    def pressure(Q):
        rho = Q[0, 0, 0]
        u = Q[1, 0, 0] / rho
        return (g - 1) * (Q[4, 0, 0] - 0.5 * rho * u * u)

    dp = (pressure(orc.rk3(ph, _acoustic_state(nx, eps, m, g, M), dt, steps))
          - pressure(orc.rk3(ph, _acoustic_state(nx, -eps, m, g, M), dt, steps))) / 2
    x = np.arange(nx) * h
    amp = np.sum(dp * np.exp(-1j * m * x)) * 2 / nx / eps
    z = -1j * sigma1(m, h) * dt / M
    P = 1 + z + z * z / 2 + z ** 3 / 6
    assert abs(amp - P ** steps) < 1e-6


def test_rk3_third_order_in_time(orc):
    """Halving dt on a fixed grid divides the error at a fixed time by ~8."""
    n = 16
    ph = orc.Physics(n=(n, n, n))
    Q0 = orc.tgv_init(ph)
    T = 0.2
    ref = orc.rk3(ph, Q0, T / 256, 256)
    errs = [np.abs(orc.rk3(ph, Q0, T / s, s) - ref).max() for s in (8, 16, 32)]
    ratios = [errs[i] / errs[i + 1] for i in range(2)]
    assert all(7.0 < r < 10.0 for r in ratios), ratios


def test_residual_points_match_full_residual(orc):
    """The sampled entry point evaluates exactly the same arithmetic."""
    n = (11, 7, 9)
    ph = orc.Physics(n=n)
    Q = synth.random_state(n[::-1], seed=3)
    R = orc.residual(ph, Q).reshape(5, -1)
    pts = synth.sample_points(n[::-1], 40, seed=1)
    Rp = orc.residual_points(ph, Q, pts)
    assert np.array_equal(Rp, R[:, pts].T)
