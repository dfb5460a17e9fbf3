"""Integrated Green's function (IGF) of the free-space Poisson equation (oracle).

Reading (the paper gives only "Poisson solve" in the bunch rest frame, sections "ImpactX" and
"Model Assumptions"; the integrated Green's function is the published method of J. Qiang et al.,
Phys. Rev. ST Accel. Beams 9, 044204 (2006)):

    Gbar(i, j, k) = (1 / (hx hy hz)) * integral over the cell centred at (i hx, j hy, k hz)
                    of dV / |r|

with (hx, hy, hz) the REST-FRAME cell (hz = gamma * lab hz).  The cell integral is the
alternating sum over the 8 cell corners of the antiderivative

    F(x,y,z) = x y ln(z+r) + y z ln(x+r) + z x ln(y+r)
               - x^2/2 atan(y z/(x r)) - y^2/2 atan(z x/(y r)) - z^2/2 atan(x y/(z r)),

r = sqrt(x^2+y^2+z^2), with every term whose prefactor is zero taken as zero
(d^3 F / dx dy dz = 1/r).  The corner formula is used only on the non-negative octant; a cell
that straddles a coordinate plane (index 0 on that axis) is folded onto [0, h/2] with weight 2,
using the evenness of 1/r.

Conditioning: the 8-corner sum cancels by a factor up to ~1e8 for far cells of elongated
rest-frame cells, which in plain float64 leaves ~1e-7 relative error in Gbar and ~1e-11 in
the field.  The oracle therefore evaluates F and the corner sum in double-double arithmetic
(oracle.dd) and rounds the cell average to float64 once, so the returned array is the cell
average of 1/r to float64 rounding.

The field's own cell averages (field_cell_average: the mean of u_a/|r|^3 over the cell, by the
2-D antiderivative H of field_antiderivative) give E' without differencing phi.

Pinned by tests/test_oracle_igf.py: unit-cube closed form 3 ln(2+sqrt3) - pi/2; scipy adaptive
cubature for anisotropic cells; 50-digit mpmath corner sums for far, elongated cells;
Gbar(d) |d| -> 1 with an O((h/d)^4) error for cubic cells.  The field kernels by
tests/test_oracle_field.py: scipy cubature, the far-field limit, the direct sum, and the exact
field of a uniformly charged box (30-digit mpmath).
"""
import numpy as np

from . import dd


def _corner_coords(n, h):
    """Corner coordinates e_0 = 0, e_m = (m - 1/2) h, m = 1..n+1, as exact double-doubles."""
    m = np.arange(n + 2, dtype=np.float64)
    c = m - 0.5
    c[0] = 0.0
    return dd.two_prod(c, np.full_like(c, h))


def antiderivative(x, y, z):
    """F(x, y, z) on double-double inputs x, y, z >= 0 (broadcast arrays)."""
    x2 = dd.mul(x, x)
    y2 = dd.mul(y, y)
    z2 = dd.mul(z, z)
    r = dd.sqrt(dd.add(dd.add(x2, y2), z2))
    xz = x[0] == 0
    yz = y[0] == 0
    zz = z[0] == 0

    def safe(a, mask):
        return np.where(mask, 1.0, a[0]), np.where(mask, 0.0, a[1])

    def zero_where(t, mask):
        return np.where(mask, 0.0, t[0]), np.where(mask, 0.0, t[1])

    xy = dd.mul(x, y)
    yzp = dd.mul(y, z)
    zx = dd.mul(z, x)
    # logarithmic terms: the argument (coord + r) is > 0 whenever the prefactor is non-zero
    t1 = zero_where(dd.mul(xy, dd.log(safe(dd.add(z, r), xz | yz))), xz | yz)
    t2 = zero_where(dd.mul(yzp, dd.log(safe(dd.add(x, r), yz | zz))), yz | zz)
    t3 = zero_where(dd.mul(zx, dd.log(safe(dd.add(y, r), zz | xz))), zz | xz)
    # arctangent terms
    t4 = zero_where(dd.mul_d(dd.mul(x2, dd.atan(dd.div(yzp, safe(dd.mul(x, r), xz)))), 0.5), xz)
    t5 = zero_where(dd.mul_d(dd.mul(y2, dd.atan(dd.div(zx, safe(dd.mul(y, r), yz)))), 0.5), yz)
    t6 = zero_where(dd.mul_d(dd.mul(z2, dd.atan(dd.div(xy, safe(dd.mul(z, r), zz)))), 0.5), zz)
    s = dd.add(dd.add(t1, t2), t3)
    s = dd.sub(s, dd.add(dd.add(t4, t5), t6))
    return s


def cell_average(nx, ny, nz, hx, hy, hz):
    """Gbar(i, j, k) for i = 0..nx, j = 0..ny, k = 0..nz; array shape (nz+1, ny+1, nx+1).

    hx, hy, hz are the rest-frame cell edges in metres; the result is in 1/m.
    """
    ex = _corner_coords(nx, hx)
    ey = _corner_coords(ny, hy)
    ez = _corner_coords(nz, hz)
    # corner grid, axis order (z, y, x)
    Z = (ez[0][:, None, None], ez[1][:, None, None])
    Y = (ey[0][None, :, None], ey[1][None, :, None])
    X = (ex[0][None, None, :], ex[1][None, None, :])
    shape = (nz + 2, ny + 2, nx + 2)
    Z = (np.broadcast_to(Z[0], shape), np.broadcast_to(Z[1], shape))
    Y = (np.broadcast_to(Y[0], shape), np.broadcast_to(Y[1], shape))
    X = (np.broadcast_to(X[0], shape), np.broadcast_to(X[1], shape))
    Fc = antiderivative(X, Y, Z)
    # triple difference over the 8 corners of each cell
    D = dd.sub((Fc[0][:, :, 1:], Fc[1][:, :, 1:]), (Fc[0][:, :, :-1], Fc[1][:, :, :-1]))
    D = dd.sub((D[0][:, 1:, :], D[1][:, 1:, :]), (D[0][:, :-1, :], D[1][:, :-1, :]))
    D = dd.sub((D[0][1:, :, :], D[1][1:, :, :]), (D[0][:-1, :, :], D[1][:-1, :, :]))
    # fold the cells that straddle a coordinate plane (index 0): weight 2 per folded axis
    w = np.ones((nz + 1, ny + 1, nx + 1))
    w[0, :, :] *= 2.0
    w[:, 0, :] *= 2.0
    w[:, :, 0] *= 2.0
    D = (D[0] * w, D[1] * w)
    vol = dd.mul(dd.two_prod(np.float64(hx), np.float64(hy)), dd.dd(np.float64(hz)))
    vol = (np.full(D[0].shape, vol[0]), np.full(D[0].shape, vol[1]))
    return dd.to_float(dd.div(D, vol))


def field_antiderivative(u, v, w):
    """H(u, v, w) = v ln(w + r) + w ln(v + r) - u atan(v w / (u r)) on double-double inputs >= 0
    (terms with a zero prefactor taken as zero): d^2 H / dv dw = 1/r, so that the cell integral
    of u/r^3 = -d(1/r)/du is minus the alternating 8-corner sum of H."""
    u2 = dd.mul(u, u)
    v2 = dd.mul(v, v)
    w2 = dd.mul(w, w)
    r = dd.sqrt(dd.add(dd.add(u2, v2), w2))
    uz = u[0] == 0
    vz = v[0] == 0
    wz = w[0] == 0

    def safe(a, mask):
        return np.where(mask, 1.0, a[0]), np.where(mask, 0.0, a[1])

    def zero_where(t, mask):
        return np.where(mask, 0.0, t[0]), np.where(mask, 0.0, t[1])

    # v ln(w + r): w + r > 0 unless v = w = 0 (then u > 0 or the term is 0 anyway)
    t1 = zero_where(dd.mul(v, dd.log(safe(dd.add(w, r), vz | (wz & uz)))), vz | (wz & uz))
    t2 = zero_where(dd.mul(w, dd.log(safe(dd.add(v, r), wz | (vz & uz)))), wz | (vz & uz))
    t3 = zero_where(dd.mul(u, dd.atan(dd.div(dd.mul(v, w), safe(dd.mul(u, r), uz)))), uz)
    return dd.sub(dd.add(t1, t2), t3)


def field_cell_average(nx, ny, nz, hx, hy, hz, axis):
    """Kbar_a(i, j, k) = (1 / (hx hy hz)) * integral over the rest-frame cell centred at
    (i hx, j hy, k hz) of u_a / |r|^3 (u_0 = x, u_1 = y, u_2 = z), for i = 0..nx, j = 0..ny,
    k = 0..nz; shape (nz+1, ny+1, nx+1).  The kernel is odd along `axis` (zero at index 0 there)
    and even along the other two, whose index-0 cells are folded with weight 2 as for Gbar.
    Evaluated as minus the 8-corner sum of field_antiderivative in double-double, rounded to
    float64 once (the corner sum cancels as that of Gbar does)."""
    ex = _corner_coords(nx, hx)
    ey = _corner_coords(ny, hy)
    ez = _corner_coords(nz, hz)
    shape = (nz + 2, ny + 2, nx + 2)
    Z = tuple(np.broadcast_to(c[:, None, None], shape) for c in ez)
    Y = tuple(np.broadcast_to(c[None, :, None], shape) for c in ey)
    X = tuple(np.broadcast_to(c[None, None, :], shape) for c in ex)
    U = (X, Y, Z)
    a = axis
    Hc = field_antiderivative(U[a], U[(a + 1) % 3], U[(a + 2) % 3])
    D = dd.sub((Hc[0][:, :, 1:], Hc[1][:, :, 1:]), (Hc[0][:, :, :-1], Hc[1][:, :, :-1]))
    D = dd.sub((D[0][:, 1:, :], D[1][:, 1:, :]), (D[0][:, :-1, :], D[1][:, :-1, :]))
    D = dd.sub((D[0][1:, :, :], D[1][1:, :, :]), (D[0][:-1, :, :], D[1][:-1, :, :]))
    w = -np.ones((nz + 1, ny + 1, nx + 1))
    for b in range(3):
        idx = [slice(None)] * 3
        idx[2 - b] = 0          # array axes are (z, y, x)
        w[tuple(idx)] *= 0.0 if b == a else 2.0
    D = (D[0] * w, D[1] * w)
    vol = dd.mul(dd.two_prod(np.float64(hx), np.float64(hy)), dd.dd(np.float64(hz)))
    vol = (np.full(D[0].shape, vol[0]), np.full(D[0].shape, vol[1]))
    return dd.to_float(dd.div(D, vol))


# ----------------------------------------------------------------------------- h-derivatives
# The kernels depend on the rest-frame cell (hx, hy, hz), which the grid geometry takes from the
# particles' box every step; the reverse sweep needs their derivatives in h.  For the cell
# average of f over the cell centred at n h, substituting r = h s (s over the unit cell around
# n) gives d/dh_b avg(f) = (1/h_b) avg(r_b df/dr_b), and integrating by parts in r_b,
#     avg(r_b df/dr_b) = (1/V) [r_b (integral of f over the face normal to b)] - avg(f),
# the bracket being the alternating sum over the two faces.  With the face integral written as
# an alternating sum over the face's corners of a 2-D antiderivative, both parts are 8-corner
# sums of one corner function C, so d/dh_b avg(f) = (fold / (V h_b)) * (8-corner sum of C),
# with the same folding of index-0 cells as the kernel itself.


def _corner_grid(nx, ny, nz, hx, hy, hz):
    """The corner coordinates (x, y, z) of the octant's cells as broadcast double-doubles."""
    ex = _corner_coords(nx, hx)
    ey = _corner_coords(ny, hy)
    ez = _corner_coords(nz, hz)
    shape = (nz + 2, ny + 2, nx + 2)
    Z = tuple(np.broadcast_to(c[:, None, None], shape) for c in ez)
    Y = tuple(np.broadcast_to(c[None, :, None], shape) for c in ey)
    X = tuple(np.broadcast_to(c[None, None, :], shape) for c in ex)
    return X, Y, Z


def _corner_sum_over_vh(Cc, fold, hx, hy, hz, hb):
    """(fold / (hx hy hz hb)) * (alternating 8-corner sum of the corner values Cc), rounded to
    float64 once; fold has the cells' shape (nz+1, ny+1, nx+1)."""
    D = dd.sub((Cc[0][:, :, 1:], Cc[1][:, :, 1:]), (Cc[0][:, :, :-1], Cc[1][:, :, :-1]))
    D = dd.sub((D[0][:, 1:, :], D[1][:, 1:, :]), (D[0][:, :-1, :], D[1][:, :-1, :]))
    D = dd.sub((D[0][1:, :, :], D[1][1:, :, :]), (D[0][:-1, :, :], D[1][:-1, :, :]))
    D = (D[0] * fold, D[1] * fold)
    den = dd.mul(dd.mul(dd.two_prod(np.float64(hx), np.float64(hy)), dd.dd(np.float64(hz))),
                 dd.dd(np.float64(hb)))
    den = (np.full(D[0].shape, den[0]), np.full(D[0].shape, den[1]))
    return dd.to_float(dd.div(D, den))


def cell_average_dh(nx, ny, nz, hx, hy, hz, b):
    """d Gbar / d h_b (b = 0, 1, 2 for hx, hy, hz) on the octant, shape (nz+1, ny+1, nx+1).

    With f = 1/r: r_b df/dr_b = -r_b^2/r^3; the face integral of 1/r is the corner sum of
    field_antiderivative H_b (d^2 H_b / dv dw = 1/r), and the cell integral of 1/r that of F,
    so the corner function is r_b H_b - F.  Even along every axis (index-0 cells folded with
    weight 2).  Identity: sum_b h_b dGbar/dh_b = -Gbar (Gbar is homogeneous of degree -1)."""
    U = _corner_grid(nx, ny, nz, hx, hy, hz)
    Fc = antiderivative(*U)
    Hb = field_antiderivative(U[b], U[(b + 1) % 3], U[(b + 2) % 3])
    Cc = dd.sub(dd.mul(U[b], Hb), Fc)
    fold = np.ones((nz + 1, ny + 1, nx + 1))
    fold[0, :, :] *= 2.0
    fold[:, 0, :] *= 2.0
    fold[:, :, 0] *= 2.0
    return _corner_sum_over_vh(Cc, fold, hx, hy, hz, (hx, hy, hz)[b])


def field_cell_average_dh(nx, ny, nz, hx, hy, hz, axis, b):
    """d Kbar_axis / d h_b on the octant, shape (nz+1, ny+1, nx+1), with Kbar_a the cell
    average of u_a/|r|^3 (field_cell_average).

    f = u_a/r^3.  The cell integral of f is minus the corner sum of H_a (field_antiderivative
    with u = u_a).  The face integral normal to b: for b = a, over (v, w), of u/r^3, whose 2-D
    antiderivative is atan(v w/(u r)); for b != a, over (u_a, u_c) (c the third axis), of
    u_a/r^3, whose antiderivative is -ln(u_c + r).  The corner function is therefore
    u_a atan(v w/(u_a r)) + H_a for b = a and -u_b ln(u_c + r) + H_a otherwise (a term with a
    zero prefactor taken as zero).  Odd along `axis`, even along the others, folded as
    Kbar_a.  Identity: sum_b h_b dKbar_a/dh_b = -2 Kbar_a (homogeneous of degree -2)."""
    U = _corner_grid(nx, ny, nz, hx, hy, hz)
    a = axis
    u, v, w = U[a], U[(a + 1) % 3], U[(a + 2) % 3]
    Ha = field_antiderivative(u, v, w)
    r = dd.sqrt(dd.add(dd.add(dd.mul(u, u), dd.mul(v, v)), dd.mul(w, w)))

    def zero_where(t, mask):
        return np.where(mask, 0.0, t[0]), np.where(mask, 0.0, t[1])

    def safe(t, mask):
        return np.where(mask, 1.0, t[0]), np.where(mask, 0.0, t[1])

    if b == a:
        uz = u[0] == 0
        t = zero_where(dd.mul(u, dd.atan(dd.div(dd.mul(v, w), safe(dd.mul(u, r), uz)))), uz)
    else:
        c = 3 - a - b
        ub, uc = U[b], U[c]
        bz = ub[0] == 0
        # u_c + r > 0 unless u_c = r = 0, where u_b = 0 too
        t = zero_where(dd.mul(ub, dd.log(safe(dd.add(uc, r), bz))), bz)
        t = (-t[0], -t[1])
    Cc = dd.add(t, Ha)
    fold = np.ones((nz + 1, ny + 1, nx + 1))
    for q in range(3):
        idx = [slice(None)] * 3
        idx[2 - q] = 0          # array axes are (z, y, x)
        fold[tuple(idx)] *= 0.0 if q == a else 2.0
    return _corner_sum_over_vh(Cc, fold, hx, hy, hz, (hx, hy, hz)[b])


def hockney_array_field(kbar, axis):
    """Place Kbar_axis in the (2nz, 2ny, 2nx) cyclic array: even along the other axes as in
    hockney_array, odd along `axis` (index t holds Kbar(t) for t < n, -Kbar(M - t) for t > n,
    and 0 at t = n, an offset no output node 0..n-1 reaches)."""
    nz, ny, nx = (s - 1 for s in kbar.shape)
    ns = (nz, ny, nx)

    def offs(n):
        M = 2 * n
        t = np.arange(M)
        return np.where(t <= n, t, M - t)

    full = kbar[np.ix_(offs(nz), offs(ny), offs(nx))].copy()
    ax = 2 - axis
    n = ns[ax]
    M = 2 * n
    sign = np.ones(M)
    sign[n + 1:] = -1.0
    sign[n] = 0.0
    shp = [1, 1, 1]
    shp[ax] = M
    return full * sign.reshape(shp)


def hockney_array(gbar):
    """Place Gbar even-symmetrically in the (2nz, 2ny, 2nx) cyclic array.

    Index t of an axis of length M = 2n holds offset t for t = 0..n and offset M - t for
    t = n+1..M-1, so the cyclic convolution with a source on nodes 0..n-1 equals the free-space
    sum for output nodes -1 (index M-1) through n.
    """
    nz, ny, nx = (s - 1 for s in gbar.shape)

    def offs(n):
        M = 2 * n
        t = np.arange(M)
        return np.where(t <= n, t, M - t)

    return gbar[np.ix_(offs(nz), offs(ny), offs(nx))]
