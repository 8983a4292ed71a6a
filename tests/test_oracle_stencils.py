"""Pins of the oracle's stencils against what the paper and the mathematics
fix (CPU only).

* The printed coefficients of equations (fd) and (sd) (golden fixture).
* Exactness on polynomials: (fd) is exact up to degree 4, (sd) up to degree
  5, the nested mixed stencil for x^a y^b with a, b <= 4; one degree more
  must fail, so the test would see a truncated stencil.
* Closed-form symbols on the periodic grid (this also pins the wrap-around
  gather and the direction <-> array-axis mapping).
* Fourth-order convergence on smooth sinusoids.
"""
import json
import math
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")


@pytest.fixture(scope="module")
def paper():
    with open(GOLDEN) as f:
        return json.load(f)


def _impulse_response(orc, order, h=1.0):
    """Weights w_s such that D f(0) = sum_s w_s f(s): apply the stencil to
    unit impulses."""
    w = []
    for s in (-2, -1, 0, 1, 2):
        f = np.zeros(5)
        f[2 + s] = 1.0
        out = orc.stencil_line(f, h, order)
        w.append(out[2])
    return np.array(w)


def test_first_derivative_coefficients_match_paper(orc, paper):
    c = paper["first_derivative"]
    want = np.array(c["numerators"], float) / np.array(c["denominators"], float)
    got = _impulse_response(orc, 1)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-15)
    # the listing's 8(f+1 - f-1) - (f+2 - f-2) over 12 h form is the same
    lst = np.array(paper["listing_first_derivative"]["weights_times_12"], float) / 12
    np.testing.assert_allclose(got, lst, rtol=0, atol=1e-15)


def test_second_derivative_coefficients_match_paper(orc, paper):
    c = paper["second_derivative"]
    want = np.array(c["numerators"], float) / np.array(c["denominators"], float)
    got = _impulse_response(orc, 2)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-15)


def test_scale_with_h(orc):
    for h in (0.1, 0.37, 2.0):
        np.testing.assert_allclose(_impulse_response(orc, 1, h),
                                   _impulse_response(orc, 1) / h, rtol=1e-15)
        np.testing.assert_allclose(_impulse_response(orc, 2, h),
                                   _impulse_response(orc, 2) / h ** 2, rtol=1e-14)


def _poly_err(orc, deg, order, h=0.1, x0=0.3, n=12):
    x = x0 + h * np.arange(n)
    f = x ** deg
    if order == 1:
        exact = deg * x ** (deg - 1) if deg > 0 else 0 * x
    else:
        exact = deg * (deg - 1) * x ** (deg - 2) if deg > 1 else 0 * x
    out = orc.stencil_line(f, h, order)
    sl = slice(2, n - 2)
    scale = max(1.0, np.abs(exact[sl]).max())
    return np.abs(out[sl] - exact[sl]).max() / scale


@pytest.mark.parametrize("deg", range(0, 5))
def test_first_derivative_exact_to_degree_4(orc, deg):
    assert _poly_err(orc, deg, 1) < 1e-12


def test_first_derivative_not_exact_at_degree_5(orc):
    assert _poly_err(orc, 5, 1) > 1e-6


@pytest.mark.parametrize("deg", range(0, 6))
def test_second_derivative_exact_to_degree_5(orc, deg):
    assert _poly_err(orc, deg, 2) < 1e-10


def test_second_derivative_not_exact_at_degree_6(orc):
    assert _poly_err(orc, 6, 2) > 1e-6


@pytest.mark.parametrize("a,b", [(a, b) for a in range(5) for b in range(5)])
def test_mixed_exact_to_degree_4_each(orc, a, b):
    hx, hy = 0.1, 0.13
    x = 0.2 + hx * np.arange(11)
    y = -0.4 + hy * np.arange(9)
    X, Y = np.meshgrid(x, y)  # [y, x]
    f = X ** a * Y ** b
    exact = (a * X ** max(a - 1, 0) if a else 0 * X) * (b * Y ** max(b - 1, 0) if b else 0 * Y)
    out = orc.mixed_plane(f, hx, hy)
    sl = (slice(2, 7), slice(2, 9))
    assert np.abs(out[sl] - exact[sl]).max() < 1e-11 * max(1.0, np.abs(exact[sl]).max())


def test_mixed_not_exact_at_degree_5(orc):
    hx, hy = 0.1, 0.13
    x = 0.2 + hx * np.arange(11)
    y = -0.4 + hy * np.arange(9)
    X, Y = np.meshgrid(x, y)
    out = orc.mixed_plane(X ** 5 * Y, hx, hy)
    exact = 5 * X ** 4
    assert np.abs(out[2:7, 2:9] - exact[2:7, 2:9]).max() > 1e-6


def sigma1(m, h):
    """Symbol of eq. (fd): D sin(m x) = sigma1 cos(m x)."""
    return (8 * math.sin(m * h) - math.sin(2 * m * h)) / (6 * h)


def sigma2(m, h):
    """Symbol of eq. (sd): D2 cos(m x) = -sigma2 cos(m x)."""
    return (2.5 - (8 / 3) * math.cos(m * h) + math.cos(2 * m * h) / 6) / h ** 2


def _grid(ph):
    nx, ny, nz = ph.n
    hx, hy, hz = ph.h
    z, y, x = np.meshgrid(np.arange(nz) * hz, np.arange(ny) * hy,
                          np.arange(nx) * hx, indexing="ij")
    return x, y, z


@pytest.mark.parametrize("d", [0, 1, 2])
def test_periodic_symbols(orc, d):
    ph = orc.Physics(n=(12, 10, 14))
    X = _grid(ph)
    h = ph.h[d]
    for m in (1, 2, 3):
        f = np.sin(m * X[d] + 0.3)
        got = orc.deriv_field(ph, f, d, 1)
        np.testing.assert_allclose(got, sigma1(m, h) * np.cos(m * X[d] + 0.3),
                                   rtol=0, atol=1e-13)
        g2 = orc.deriv_field(ph, f, d, 2)
        np.testing.assert_allclose(g2, -sigma2(m, h) * f, rtol=0, atol=1e-12)
        # the other two directions see a constant: exactly zero for (fd)
        for e in range(3):
            if e != d:
                assert np.all(orc.deriv_field(ph, f, e, 1) == 0.0)


@pytest.mark.parametrize("di,dk", [(0, 1), (1, 0), (0, 2), (2, 0), (1, 2), (2, 1)])
def test_periodic_mixed_symbol(orc, di, dk):
    ph = orc.Physics(n=(12, 10, 14))
    X = _grid(ph)
    mi, mk = 2, 1
    f = np.sin(mi * X[di]) * np.sin(mk * X[dk])
    got = orc.mixed_field(ph, f, di, dk)
    want = sigma1(mi, ph.h[di]) * sigma1(mk, ph.h[dk]) * np.cos(mi * X[di]) * np.cos(mk * X[dk])
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-13)


def test_fourth_order_convergence(orc):
    errs1, errs2, errsm = [], [], []
    for n in (16, 32, 64, 128):
        ph = orc.Physics(n=(n, 5, 6))
        x = np.arange(n) * ph.h[0]
        f = np.broadcast_to(np.exp(np.sin(x)), (6, 5, n))
        d1 = orc.deriv_field(ph, f, 0, 1)[0, 0]
        d2 = orc.deriv_field(ph, f, 0, 2)[0, 0]
        e = np.exp(np.sin(x))
        errs1.append(np.abs(d1 - np.cos(x) * e).max())
        errs2.append(np.abs(d2 - (np.cos(x) ** 2 - np.sin(x)) * e).max())
        ph2 = orc.Physics(n=(n, n, 5))
        X = _grid(ph2)
        g = np.sin(X[0]) * np.exp(np.cos(X[1]))
        dm = orc.mixed_field(ph2, g, 0, 1)
        errsm.append(np.abs(dm + np.cos(X[0]) * np.sin(X[1]) * np.exp(np.cos(X[1]))).max())
    for errs in (errs1, errs2, errsm):
        rates = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
        assert all(3.8 < r < 4.3 for r in rates[1:]), (errs, rates)
