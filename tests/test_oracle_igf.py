"""Pins of the oracle's integrated Green's function (cell average of 1/|r|)."""
import mpmath as mp
import numpy as np
import pytest
from scipy import integrate

from oracle import igf


def test_unit_cube_closed_form():
    # average of 1/r over the unit cube centred on the origin = 3 ln(2 + sqrt 3) - pi/2
    g = igf.cell_average(1, 1, 1, 1.0, 1.0, 1.0)
    exact = 3.0 * np.log(2.0 + np.sqrt(3.0)) - np.pi / 2.0
    assert abs(g[0, 0, 0] - exact) < 2e-16 * exact
    # scaling: Gbar(0) h = const for a cube of edge h
    g2 = igf.cell_average(1, 1, 1, 0.25, 0.25, 0.25)
    assert abs(g2[0, 0, 0] * 0.25 - exact) < 4e-16 * exact


def test_far_field_order_h4_for_cubes():
    g = igf.cell_average(16, 16, 16, 1.0, 1.0, 1.0)
    # along an axis and along the diagonal the cell average tends to 1/|d| with an
    # O((h/d)^4) error (the h^2 term vanishes because 1/r is harmonic)
    for d0 in (4, 8):
        e1 = abs(g[0, 0, d0] * d0 - 1.0)
        e2 = abs(g[0, 0, 2 * d0] * 2 * d0 - 1.0)
        assert 12.0 < e1 / e2 < 20.0
        r1 = np.sqrt(3.0) * d0
        e1 = abs(g[d0, d0, d0] * r1 - 1.0)
        e2 = abs(g[2 * d0, 2 * d0, 2 * d0] * 2 * r1 - 1.0)
        assert 10.0 < e1 / e2 < 22.0
    assert abs(g[0, 0, 8] * 8 - 1.0) < 1e-4


@pytest.mark.parametrize("cell", [(2, 1, 3), (0, 3, 1), (5, 0, 0), (1, 1, 1)])
def test_anisotropic_against_scipy_cubature(cell):
    h = (1.0, 1.5, 40.0)
    i, j, k = cell
    g = igf.cell_average(6, 6, 6, *h)

    def lims(m, hh):
        return (m - 0.5) * hh, (m + 0.5) * hh

    (x0, x1), (y0, y1), (z0, z1) = lims(i, h[0]), lims(j, h[1]), lims(k, h[2])

    # integrate z analytically (asinh), x and y by adaptive quadrature
    def inner(y, x):
        rho = np.hypot(x, y)
        return np.arcsinh(z1 / rho) - np.arcsinh(z0 / rho)

    val, err = integrate.dblquad(inner, x0, x1, y0, y1, epsabs=0, epsrel=1e-12)
    ref = val / (h[0] * h[1] * h[2])
    assert abs(g[k, j, i] - ref) < 1e-10 * ref


def _mp_cell(i, j, k, h):
    mp.mp.dps = 60

    def F(x, y, z):
        r = mp.sqrt(x * x + y * y + z * z)
        s = mp.mpf(0)
        if x and y:
            s += x * y * mp.log(z + r)
        if y and z:
            s += y * z * mp.log(x + r)
        if z and x:
            s += z * x * mp.log(y + r)
        if x:
            s -= x * x / 2 * mp.atan(y * z / (x * r))
        if y:
            s -= y * y / 2 * mp.atan(z * x / (y * r))
        if z:
            s -= z * z / 2 * mp.atan(x * y / (z * r))
        return s

    def edges(m, hh):
        hh = mp.mpf(hh)
        return (mp.mpf(0), hh / 2) if m == 0 else ((m - mp.mpf(0.5)) * hh, (m + mp.mpf(0.5)) * hh)

    ex, ey, ez = edges(i, h[0]), edges(j, h[1]), edges(k, h[2])
    s = mp.mpf(0)
    for a in range(2):
        for b in range(2):
            for c in range(2):
                s += (-1) ** (3 - a - b - c) * F(ex[a], ey[b], ez[c])
    w = (2 if i == 0 else 1) * (2 if j == 0 else 1) * (2 if k == 0 else 1)
    return s * w / (mp.mpf(h[0]) * mp.mpf(h[1]) * mp.mpf(h[2]))


@pytest.mark.parametrize("h", [(1.0, 1.0, 1.0), (1.0, 1.0, 200.0), (0.7, 1.3, 7800.0)])
def test_far_cells_against_50_digit_corner_sums(h):
    n = 40
    g = igf.cell_average(n, n, n, *h)
    cells = [(0, 0, 0), (1, 0, 0), (0, 0, 1), (n, n, n), (n, 0, 0), (0, n, 0), (0, 0, n),
             (3, 37, 7), (n, n, 1), (17, 33, n), (1, 1, 1)]
    for (i, j, k) in cells:
        ref = _mp_cell(i, j, k, h)
        assert abs((mp.mpf(float(g[k, j, i])) - ref) / ref) < 2.5e-16


def test_hockney_placement_is_even():
    g = igf.cell_average(4, 3, 5, 1.0, 2.0, 3.0)
    G = igf.hockney_array(g)
    assert G.shape == (10, 6, 8)
    for ax, M in ((0, 10), (1, 6), (2, 8)):
        t = np.arange(1, M)
        assert np.array_equal(np.take(G, t, axis=ax), np.take(G, M - t, axis=ax))
    assert G[5, 3, 4] == g[5, 3, 4]
