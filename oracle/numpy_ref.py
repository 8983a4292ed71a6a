"""Second, independent evaluation of R(Q) with NumPy ``np.roll`` stencils.

TEST INFRASTRUCTURE ONLY (see the package docstring).  It exists to
cross-check the C oracle on small grids: it is written from the same
equations of the methodology section of arXiv:1709.09713 but in a different
arithmetic form, so that a slip in either implementation shows up as a
disagreement far above rounding:

* first derivatives use the 8(f[+1]-f[-1]) - (f[+2]-f[-2]) over 12h form of
  the Fortran listing of the baseline algorithm instead of eq. (fd)'s
  coefficient form;
* the viscous bracket is simplified by hand to
  lap(u_i) + (1/3) d/dx_i (div u), the dissipation to
  sum_ij du_i/dx_j (du_i/dx_j + du_j/dx_i) - (2/3) div^2;
* whole-field vectorised operations instead of per-point gathers.

Arrays are indexed [z, y, x]; direction d = 0 is x (numpy axis 2).
"""
from __future__ import annotations

import numpy as np

_AX = {0: 2, 1: 1, 2: 0}


def _sh(f, d, s):
    """f evaluated at the point shifted by +s along direction d."""
    return np.roll(f, -s, axis=_AX[d])


def d1(f, d, h):
    return (8.0 * (_sh(f, d, 1) - _sh(f, d, -1))
            - (_sh(f, d, 2) - _sh(f, d, -2))) / (12.0 * h[d])


def d2(f, d, h):
    return (-(_sh(f, d, 2) + _sh(f, d, -2))
            + 16.0 * (_sh(f, d, 1) + _sh(f, d, -1)) - 30.0 * f) / (12.0 * h[d] ** 2)


def residual(Q, h, gamma, prandtl, reynolds, mach):
    rho, m, E = Q[0], Q[1:4], Q[4]
    u = m / rho
    p = (gamma - 1.0) * (E - 0.5 * (m * u).sum(axis=0))
    T = gamma * mach ** 2 * p / rho
    inv_re = 0.0 if np.isinf(reynolds) else 1.0 / reynolds
    kappa = inv_re / ((gamma - 1.0) * mach ** 2 * prandtl)

    g = np.array([[d1(u[i], j, h) for j in range(3)] for i in range(3)])
    div = g[0, 0] + g[1, 1] + g[2, 2]

    R = np.empty_like(Q)
    R[0] = -0.5 * sum(d1(m[j], j, h) + rho * g[j, j] + u[j] * d1(rho, j, h)
                      for j in range(3))
    V = []
    for i in range(3):
        lap = sum(d2(u[i], j, h) for j in range(3))
        graddiv = d2(u[i], i, h) + sum(d1(d1(u[k], k, h), i, h)
                                       for k in range(3) if k != i)
        V.append(lap + graddiv / 3.0)
        conv = sum(d1(m[i] * u[j], j, h) + m[i] * g[j, j]
                   + u[j] * d1(m[i], j, h) for j in range(3))
        R[1 + i] = -0.5 * conv - d1(p, i, h) + inv_re * V[i]
    phi = sum(g[i, j] * (g[i, j] + g[j, i]) for i in range(3)
              for j in range(3)) - (2.0 / 3.0) * div ** 2
    conv = sum(d1(E * u[j], j, h) + E * g[j, j] + u[j] * d1(E, j, h)
               for j in range(3))
    R[4] = (-0.5 * conv - sum(d1(p * u[j], j, h) for j in range(3))
            + inv_re * (sum(u[i] * V[i] for i in range(3)) + phi)
            + kappa * sum(d2(T, j, h) for j in range(3)))
    return R


def energy_leak(Q, h, reynolds):
    """sum over the grid of the viscous part of R_E that the discrete
    operators do not telescope: (1/Re) [sum_ij u_i.(D2_j - D_j D_j) u_i
    + (1/3) sum_i u_i.(D2_i - D_i D_i) u_i].  Mass, momentum and the rest of
    the energy residual sum to zero exactly in exact arithmetic."""
    u = Q[1:4] / Q[0]
    leak = 0.0
    for i in range(3):
        for j in range(3):
            leak += np.sum(u[i] * (d2(u[i], j, h) - d1(d1(u[i], j, h), j, h)))
        leak += np.sum(u[i] * (d2(u[i], i, h) - d1(d1(u[i], i, h), i, h))) / 3.0
    return leak / reynolds
