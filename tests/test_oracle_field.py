"""Pins of the oracle's direct-field solve (the field's own integrated Green's function).

* Cell averages of u_a/|r|^3 against scipy adaptive cubature, for anisotropic cells, folded
  cells on the coordinate planes and the odd kernel's zero plane.
* Far field: Kbar -> x/R^3 with an O((h/R)^2) error.
* The zero-padded FFT convolution with the odd/even kernel array against the direct sum.
* A uniformly charged ellipsoid: inside, both field paths give the linear closed form
  E_i = rho n_i x_i / eps0 with the depolarisation factors n_i (quadrature; 1/3 for a sphere).
* A uniformly charged box made of whole cells, whose exact field at every node follows from
  the box's own 8-corner antiderivative sum, evaluated independently in 30-digit mpmath: the
  direct-field solve reproduces it to rounding, while -grad phi by centred differences of the
  potential solve is off by O(h^2).
"""
import mpmath
import numpy as np
import pytest
from scipy import integrate

from ellipsoid_math import depolarisation
from oracle import igf, pic

H = (1.0, 0.7, 2.3)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_field_cell_average_against_cubature(axis):
    hx, hy, hz = H
    K = igf.field_cell_average(4, 4, 4, hx, hy, hz, axis)
    h = np.array(H)
    for (i, j, k) in ((1, 0, 0), (0, 1, 0), (0, 0, 1), (2, 1, 3), (0, 2, 1), (3, 3, 2)):
        c = np.array([i, j, k]) * h
        lo, hi = c - h / 2, c + h / 2

        def f(x, y, z):
            return (x, y, z)[axis] / (x * x + y * y + z * z) ** 1.5

        if (i, j, k)[axis] == 0:   # the odd kernel vanishes on its own zero plane
            assert K[k, j, i] == 0.0
            continue
        val, _ = integrate.nquad(f, [[lo[0], hi[0]], [lo[1], hi[1]], [lo[2], hi[2]]],
                                 opts={"epsabs": 0, "epsrel": 1e-12})
        ref = val / np.prod(h)
        assert abs(K[k, j, i] - ref) < 1e-13 * abs(ref), (axis, i, j, k)


def test_far_field_limit():
    # cubic cells: Kbar_x (i, j, k) R^3 / x -> 1 with an O((h/R)^2) error
    K = igf.field_cell_average(40, 2, 2, 1.0, 1.0, 1.0, 0)
    err = [abs(K[1, 1, i] * (i * i + 2) ** 1.5 / i - 1.0) for i in (5, 10, 20, 40)]
    for e1, e2 in zip(err, err[1:]):
        assert e2 < e1 / 3.0    # quadratic decay: about 4x per doubling of R
    assert err[-1] < 1e-3


def test_fft_convolution_equals_the_direct_sum():
    rng = np.random.default_rng(3)
    nx, ny, nz = 6, 5, 7
    Q = rng.standard_normal((nz, ny, nx))
    ks = [igf.field_cell_average(nx, ny, nz, *H, a) for a in range(3)]
    E = pic.solve_field(Q, ks) * (4.0 * np.pi * pic.EPS0)
    ref = np.zeros_like(E)
    sign = [(-1, 1, 1), (1, -1, 1), (1, 1, -1)]   # parity of Kbar_a under (x, y, z) -> -(.)
    for a in range(3):
        for k in range(nz):
            for j in range(ny):
                for i in range(nx):
                    s = 0.0
                    for m in range(nz):
                        for l in range(ny):
                            for p in range(nx):
                                di, dj, dk = i - p, j - l, k - m
                                v = ks[a][abs(dk), abs(dj), abs(di)]
                                for d, sg in zip((di, dj, dk), sign[a]):
                                    if d < 0 and sg < 0:
                                        v = -v
                                s += Q[m, l, p] * v
                    ref[a, k, j, i] = s
    assert np.abs(E - ref).max() < 1e-13 * np.abs(ref).max()


def _box_field_mp(p, lo, hi, axis):
    """integral over the box [lo, hi] of (p - r')_axis / |p - r'|^3 dV', in 30-digit mpmath,
    by splitting the box at p into sub-boxes with p at a corner and summing the corner formula
    of the antiderivative H(u, v, w) = v ln(w + r) + w ln(v + r) - u atan(v w/(u r))."""
    mpmath.mp.dps = 30

    def Hm(u, v, w):
        r = mpmath.sqrt(u * u + v * v + w * w)
        t = mpmath.mpf(0)
        if v != 0 and (w != 0 or u != 0):
            t += v * mpmath.log(w + r)
        if w != 0 and (v != 0 or u != 0):
            t += w * mpmath.log(v + r)
        if u != 0:
            t -= u * mpmath.atan(v * w / (u * r))
        return t

    b, c = (axis + 1) % 3, (axis + 2) % 3
    total = mpmath.mpf(0)
    # per axis: the distance interval(s) from p, with the sign of the offset p - r'
    pieces = []
    for q in range(3):
        a0, a1 = mpmath.mpf(lo[q]) - p[q], mpmath.mpf(hi[q]) - p[q]
        if a0 >= 0:
            pieces.append([(a0, a1, -1)])            # r' above p: offset p - r' < 0
        elif a1 <= 0:
            pieces.append([(-a1, -a0, 1)])
        else:
            pieces.append([(mpmath.mpf(0), -a0, 1), (mpmath.mpf(0), a1, -1)])
    for px in pieces[0]:
        for py in pieces[1]:
            for pz in pieces[2]:
                iv = (px, py, pz)
                s = mpmath.mpf(0)
                for cu in (0, 1):
                    for cv in (0, 1):
                        for cw in (0, 1):
                            u = iv[axis][cu]
                            v = iv[b][cv]
                            w = iv[c][cw]
                            sg = (-1) ** (cu + cv + cw + 1)
                            s += sg * Hm(u, v, w)
                # integral of u/r^3 over the sub-box (distances >= 0) is minus the corner sum
                total += iv[axis][2] * (-s)
    return total


def test_uniformly_charged_box_field_is_exact():
    nx, ny, nz = 12, 10, 14
    hx, hy, hz = H
    cells = ((3, 8), (2, 7), (4, 10))           # whole cells [i0, i1) on each axis
    Q = np.zeros((nz, ny, nx))
    Q[cells[2][0]:cells[2][1], cells[1][0]:cells[1][1], cells[0][0]:cells[0][1]] = 1.0
    rho = 1.0 / (hx * hy * hz)
    E = pic.solve_field(Q, [igf.field_cell_average(nx, ny, nz, hx, hy, hz, a) for a in range(3)])
    phi = pic.solve(Q, igf.cell_average(nx, ny, nz, hx, hy, hz))
    geom = pic.Geometry(np.zeros(3), np.array(H), np.array(H))
    Efd = pic.field(phi, geom)
    h = np.array(H)
    lo = np.array([cells[0][0], cells[1][0], cells[2][0]]) * h - h / 2
    hi = np.array([cells[0][1], cells[1][1], cells[2][1]]) * h - h / 2
    rng = np.random.default_rng(7)
    nodes = [(0, 0, 0), (5, 4, 6), (3, 2, 4), (11, 9, 13), (7, 6, 9)]
    nodes += [tuple(int(v) for v in rng.integers(0, (nx, ny, nz))) for _ in range(20)]
    scale = np.abs(E).max()
    err_direct = err_fd = 0.0
    for (i, j, k) in nodes:
        p = [mpmath.mpf(i * hx), mpmath.mpf(j * hy), mpmath.mpf(k * hz)]
        for a in range(3):
            ref = float(_box_field_mp(p, lo, hi, a) * rho / (4 * mpmath.pi * pic.EPS0))
            err_direct = max(err_direct, abs(E[a, k, j, i] - ref))
            err_fd = max(err_fd, abs(Efd[a, k, j, i] - ref))
    assert err_direct < 1e-13 * scale
    assert err_fd > 1e-4 * scale      # the centred differences' O(h^2) error, removed above


def test_centred_differences_converge_to_the_direct_field():
    # a smooth charge (cell integrals of a Gaussian): -grad phi by centred differences differs
    # from the direct field by the differencing error, O(h^2): about 4x less per grid doubling
    from scipy.special import erf
    sig = np.array([1.0, 0.8, 1.6])
    diffs = []
    for n in (16, 32):
        h = 8 * sig / (n - 1)
        o = -4 * sig

        def cellint(a):
            x = o[a] + np.arange(n) * h[a]
            s = sig[a] * np.sqrt(2)
            return 0.5 * (erf((x + h[a] / 2) / s) - erf((x - h[a] / 2) / s))

        Q = cellint(2)[:, None, None] * cellint(1)[None, :, None] * cellint(0)[None, None, :]
        Ed = pic.solve_field(Q, [igf.field_cell_average(n, n, n, *h, a) for a in range(3)])
        Ef = pic.field(pic.solve(Q, igf.cell_average(n, n, n, *h)), pic.Geometry(o, h, h))
        diffs.append(np.abs(Ed - Ef).max() / np.abs(Ef).max())
    assert 3.5 < diffs[0] / diffs[1] < 4.5
    assert diffs[1] < 1e-2


def test_depolarisation_factors_of_a_sphere_and_their_sum():
    assert np.allclose(depolarisation((2.0, 2.0, 2.0)), 1.0 / 3.0, rtol=1e-10, atol=0)
    assert abs(depolarisation((12.0, 9.0, 30.0)).sum() - 1.0) < 1e-10


def test_uniform_ellipsoid_has_the_linear_interior_field():
    # The field inside a uniformly charged ellipsoid is E_i = rho n_i x_i / eps0 (the
    # Kurth-like beam of a linear space-charge force). The charge per cell comes from 10^3
    # sub-points in the cells the surface may cut, so only that staircase separates the
    # grid solution from the closed form: about 4e-5 of the largest interior field here, while
    # a swapped axis, a lost 4 pi or a wrong sign is off by 10 % or more.
    nx = ny = nz = 40
    h = np.array(H)
    semi = np.array([12.0, 9.0, 30.0])
    ctr = np.array([20.0, 14.0, 46.0])
    ax = [np.arange(m) * h[a] for a, m in enumerate((nx, ny, nz))]
    Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    u = [(X - ctr[0]) / semi[0], (Y - ctr[1]) / semi[1], (Z - ctr[2]) / semi[2]]
    f = u[0] ** 2 + u[1] ** 2 + u[2] ** 2
    frac = (f < 1.0).astype(float)
    # cells whose centre lies within a cell diagonal (in scaled units) of the surface
    band = np.abs(np.sqrt(f) - 1.0) < 1.5 * np.linalg.norm(h / semi)
    sub = (np.arange(10) + 0.5) / 10 - 0.5
    sz, sy, sx = np.meshgrid(sub * h[2], sub * h[1], sub * h[0], indexing="ij")
    for k, j, i in zip(*np.nonzero(band)):
        p = (X[k, j, i] + sx - ctr[0]) / semi[0], (Y[k, j, i] + sy - ctr[1]) / semi[1], \
            (Z[k, j, i] + sz - ctr[2]) / semi[2]
        frac[k, j, i] = np.mean(p[0] ** 2 + p[1] ** 2 + p[2] ** 2 < 1.0)
    rho = 1.0
    Q = rho * frac * np.prod(h)
    E = pic.solve_field(Q, [igf.field_cell_average(nx, ny, nz, *h, a) for a in range(3)])
    Efd = pic.field(pic.solve(Q, igf.cell_average(nx, ny, nz, *h)),
                    pic.Geometry(np.zeros(3), h, h))
    n_i = depolarisation(semi)
    inner = f < 0.5 ** 2
    scale = rho * max(n_i * semi) / pic.EPS0
    for a, (g, c) in enumerate(zip((X, Y, Z), ctr)):
        ref = rho * n_i[a] * (g - c) / pic.EPS0
        assert np.abs(E[a][inner] - ref[inner]).max() < 3e-4 * scale, a
        # the potential is quadratic there, so centred differences are exact up to the staircase
        assert np.abs(Efd[a][inner] - ref[inner]).max() < 3e-4 * scale, a
