"""Closed forms that the tests compare the oracle and the HIP path with.
Each is derived from the paper's equations by hand, not computed by either
implementation."""
import math

import numpy as np


# (n, length, gamma, prandtl, reynolds, mach); the second case has unequal
# spacings, Pr != 1 and gamma, M far from the TGV values, so a slip in any
# factor of kappa or of the equation of state changes R_E.
HEAT_CASES = [
    ((16, 16, 16), (2 * math.pi,) * 3, 1.4, 0.71, 1600.0, 0.1),
    ((12, 18, 10), (2 * math.pi, 3 * math.pi, 1.5 * math.pi), 1.67, 1.3, 400.0, 0.3),
]


def heat_mode_expected(case, d, m, eps, energy):
    """Closed-form residual of ``synth.resting_density_mode``: the fluid is at
    rest (u = 0) at uniform pressure p = (gamma-1) rho E (eq. pinprimitive),
    so every convective, pressure and viscous term vanishes and only heat
    conduction remains (methodology section, last term of the energy
    equation): R_E = kappa sum_j D2_j T with kappa = 1/((gamma-1) M^2 Pr Re).
    T = gamma M^2 p / rho (eq. Tinprimitive) = gamma M^2 p (1 + eps cos theta),
    and the periodic symbol of eq. (sd) gives D2 cos theta = -sigma2 cos theta."""
    n, length, g, pr, re, mach = case
    kappa = 1.0 / ((g - 1.0) * mach ** 2 * pr * re)
    p = (g - 1.0) * energy
    h = length[d] / n[d]
    th = 2 * math.pi * m / n[d]
    s2 = (2.5 - (8 / 3) * math.cos(th) + math.cos(2 * th) / 6) / h ** 2
    shape = n[::-1]
    idx = np.arange(n[d]) * th
    bshape = [1, 1, 1]
    bshape[2 - d] = n[d]
    cos = np.broadcast_to(np.cos(idx).reshape(bshape), shape)
    return -kappa * g * mach ** 2 * p * eps * s2 * cos
