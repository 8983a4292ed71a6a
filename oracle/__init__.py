"""FP64 CPU oracle for the compressible Navier-Stokes residual + RK3 path.

TEST INFRASTRUCTURE ONLY.  The test suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package; the product
package never does, and this package imports nothing from it.

``ns_oracle.c`` is the plain C definition (every function cites the passage of
arXiv:1709.09713 it follows); this module only marshals NumPy arrays to it
through ctypes.  ``numpy_ref`` is a second, independent NumPy evaluation used
to cross-check the C code on small grids.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ns_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

TWO_PI = 2.0 * math.pi


def build(force: bool = True) -> str:
    """Compile ``ns_oracle.c`` into ``liboracle.so`` (gcc, FP64, no FMA
    contraction, OpenMP over z-planes)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
             "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = ctypes.CDLL(_LIB_PATH)
        d, i, p = ctypes.c_double, ctypes.c_int, ctypes.c_void_p
        i64 = ctypes.c_int64
        L.orc_d1.restype = d
        L.orc_d1.argtypes = [d, d, d, d, d]
        L.orc_d2.restype = d
        L.orc_d2.argtypes = [d, d, d, d, d, d]
        L.orc_stencil_line.argtypes = [p, i, d, i, p]
        L.orc_mixed_plane.argtypes = [p, i, i, d, d, p]
        L.orc_deriv_field.argtypes = [i, i, i, d, d, d, p, i, i, p]
        L.orc_mixed_field.argtypes = [i, i, i, d, d, d, p, i, i, p]
        L.orc_residual.argtypes = [i, i, i, d, d, d, d, d, d, d, p, p]
        L.orc_residual_points.argtypes = [i, i, i, d, d, d, d, d, d, d, p,
                                          i64, p, p]
        L.orc_rk3.argtypes = [i, i, i, d, d, d, d, d, d, d, d, i, p]
        L.orc_tgv_init.argtypes = [i, i, i, d, d, d, d, d, p]
        L.orc_diagnostics.argtypes = [i, i, i, d, d, d, d, d, d, d, p, p]
        for f in ("orc_stencil_line", "orc_mixed_plane", "orc_deriv_field",
                  "orc_mixed_field", "orc_residual", "orc_residual_points",
                  "orc_rk3", "orc_tgv_init", "orc_diagnostics"):
            getattr(L, f).restype = None
        _lib = L
    return _lib


@dataclass(frozen=True)
class Physics:
    """Grid and non-dimensional parameters (results section: Re = 1600,
    Pr = 0.71, M = 0.1, gamma = 1.4 on [0, 2 pi]^3)."""
    n: tuple = (16, 16, 16)
    length: tuple = (TWO_PI, TWO_PI, TWO_PI)
    gamma: float = 1.4
    prandtl: float = 0.71
    reynolds: float = 1600.0
    mach: float = 0.1

    @property
    def h(self):
        return tuple(L / n for L, n in zip(self.length, self.n))

    @property
    def npoints(self) -> int:
        return self.n[0] * self.n[1] * self.n[2]

    def args(self):
        return (*self.n, *self.length, self.gamma, self.prandtl,
                self.reynolds, self.mach)


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data


def _state_shape(ph: Physics):
    nx, ny, nz = ph.n
    return (5, nz, ny, nx)


def stencil_line(f, h: float, order: int):
    """Apply eq. (fd) (order 1) or eq. (sd) (order 2) at interior points
    2..n-3 of a plain 1-D array; NaN elsewhere."""
    f, fp = _f64(f)
    out = np.full_like(f, np.nan)
    lib().orc_stencil_line(fp, f.size, h, order, out.ctypes.data)
    return out


def mixed_plane(f, hx: float, hy: float):
    """Nested D_x(D_y f) at interior points of a plain 2-D array f[y, x]."""
    f, fp = _f64(f)
    ny, nx = f.shape
    out = np.full_like(f, np.nan)
    lib().orc_mixed_plane(fp, nx, ny, hx, hy, out.ctypes.data)
    return out


def deriv_field(ph: Physics, f, d: int, order: int):
    """Periodic first/second derivative of a grid function f[z, y, x] along
    direction d (0 = x)."""
    f, fp = _f64(f)
    out = np.empty_like(f)
    lib().orc_deriv_field(*ph.n, *ph.length, fp, d, order, out.ctypes.data)
    return out


def mixed_field(ph: Physics, f, di: int, dk: int):
    """Periodic nested mixed derivative D_di(D_dk f)."""
    f, fp = _f64(f)
    out = np.empty_like(f)
    lib().orc_mixed_field(*ph.n, *ph.length, fp, di, dk, out.ctypes.data)
    return out


def tgv_init(ph: Physics):
    """Taylor-Green vortex state Q[5, nz, ny, nx] (results section)."""
    Q = np.empty(_state_shape(ph))
    lib().orc_tgv_init(*ph.n, *ph.length, ph.gamma, ph.mach, Q.ctypes.data)
    return Q


def residual(ph: Physics, Q):
    """R(Q) on the whole grid, shape [5, nz, ny, nx]."""
    Q, qp = _f64(Q)
    assert Q.shape == _state_shape(ph)
    R = np.empty_like(Q)
    lib().orc_residual(*ph.args(), qp, R.ctypes.data)
    return R


def residual_points(ph: Physics, Q, points):
    """R(Q) at linear point indices ``points``; returns [npoints, 5]."""
    Q, qp = _f64(Q)
    assert Q.shape == _state_shape(ph)
    pts = np.ascontiguousarray(points, dtype=np.int64)
    out = np.empty((pts.size, 5))
    lib().orc_residual_points(*ph.args(), qp, pts.size, pts.ctypes.data,
                              out.ctypes.data)
    return out


def rk3(ph: Physics, Q, dt: float, nsteps: int):
    """Advance a copy of Q by nsteps low-storage RK3 steps."""
    Q = np.array(Q, dtype=np.float64, order="C", copy=True)
    assert Q.shape == _state_shape(ph)
    lib().orc_rk3(*ph.args(), dt, nsteps, Q.ctypes.data)
    return Q


DIAG_NAMES = ("mass", "momentum_x", "momentum_y", "momentum_z", "energy",
              "kinetic_energy", "enstrophy", "dissipation")


def diagnostics(ph: Physics, Q):
    """Eight FP64 diagnostics (see ``orc_diagnostics``) as a dict."""
    Q, qp = _f64(Q)
    assert Q.shape == _state_shape(ph)
    out = np.empty(8)
    lib().orc_diagnostics(*ph.args(), qp, out.ctypes.data)
    return dict(zip(DIAG_NAMES, out.tolist()))

