"""Reverse sweep (discrete adjoint) of the oracle's tracking (oracle; test infrastructure).

Gradients of J = sum_k w_k m_k, m = (sigma_x, sigma_y, eps_x, eps_y) of the final beam, with
respect to the thin-quad strengths k_j, the initial coordinates X0 and, through X0 = L xi with
L the Cholesky factor, the initial second-moment matrix Sigma0.

Reading (the paper gives no differentiation; this is the project's addition): the gradient is
that of the tracked map, whose grid geometry follows the particles: every step the box is the
min / max of the kick-point positions, h_a = (max_a - min_a)/(n_a - 3.5) and
origin_a = min_a - 1.25 h_a.  The map is smooth almost everywhere (CIC weights have kinks at
nodes, TSC weights at cell boundaries in the second derivative only, and the box changes its
extreme particle on a set of measure zero).  With per-step geometries passed in (`geoms`) the
geometry is frozen instead and its terms below are left out.  The adjoint of each linear
operation is its transpose:

* drift l:        lam_px += l lam_x, lam_py += l lam_y, lam_delta += (l/gamma^2) lam_z
* thin quad k:    lam_x -= k lam_px, lam_y += k lam_py;   dJ/dk += sum(-x lam_px + y lam_py)
* space-charge kick over L, with a_i = (C L lam_px, C L lam_py, gamma C L lam_delta):
    direct (gather weights)    lam_r,i += sum_n grad W(r_i - r_n) (a_i . E'_n)
    through the charge         e_n = sum_i W(r_i - r_n) a_i              (vector deposit)
                               psi = -sum_c D_c^T e_c on nodes -1..n_a  (D_c: centred difference)
                               chi = 1/(4 pi eps0) Gbar * psi on nodes 0..n_a-1
                               lam_r,i += q_m sum_n grad W(r_i - r_n) chi_n
  grad W is taken with respect to the lab position (du/dx = 1/h).

* the geometry (geometry_adjoint): with g_i the position gradient through the weights above
  (direct + through the charge) and u_i = (x_i - origin)/h,
    dJ/dorigin_a = -sum_i g_i,a,   dJ/dh_a += -sum_i g_i,a u_i,a            (weights)
    dJ/dh'_b    += -sum_n e_b(n) E'_b(n) / h'_b                            (centred difference)
    dJ/dh'_b    += sum_n Q_n (dGbar/dh'_b * psi)_n / (4 pi eps0)           (Green's function)
  (direct field: dJ/dh'_b = sum_a sum_n e_a(n) (dKbar_a/dh'_b * Q)(n) / (4 pi eps0)), with the
  rest-frame cell h' = (hx, hy, gamma hz) and the kernels' h-derivatives of igf; then through
  h_a = (max_a - min_a)/(n_a - 3.5), origin_a = min_a - 1.25 h_a onto the kick-point
  coordinate of the particle that attains the min (the first one, as numpy's argmin) and of
  the one that attains the max
* thick quadrupole half map M(k) per plane: lam <- M^T lam; dJ/dk += lam_after . (dM/dk) X_before
  (adjoint_elements, lattices of Drift / Quad / thin elements cut into slices)
* with the direct field (Problem.direct_field) the charge's adjoint is chi = -1/(4 pi eps0)
  sum_a Kbar_a * e_a (solve_field_T: the field kernels are odd along their own axis), with no
  difference operator

Pinned by tests/test_oracle_adjoint.py: dot-product tests of every transposed operation,
central finite differences on small beams with space charge (thin lattices and lattices of
thick elements), of the tracking with the geometry following the particles and with it frozen, the closed-form gradient of the zero-current (linear) map, the
k-derivative of the quadrupole matrix against central differences and its k -> 0 limit, and
the transposed field solve by a dot product and central differences with the direct field.
"""
import numpy as np

from .constants import EPS0
from . import igf, pic


# ----------------------------------------------------------------------------- shapes

def shape_weights_and_derivs(u, shape):
    """(idx, w, dw/du) along one axis, each of shape (S, n)."""
    idx, w = pic.shape_weights(u, shape)
    if shape == 1:
        dw = np.stack([-np.ones_like(u), np.ones_like(u)])
    else:
        d = u - np.floor(u + 0.5)
        dw = np.stack([-(0.5 - d), -2.0 * d, 0.5 + d])
    return idx, w, dw


def _stencil_grad(X, geom, prob):
    """Flattened node index, weight and the three components of grad W (lab units)."""
    nx, ny, nz = prob.nodes
    ix, wx, dx = shape_weights_and_derivs((X[0] - geom.origin[0]) / geom.h[0], prob.shape)
    iy, wy, dy = shape_weights_and_derivs((X[2] - geom.origin[1]) / geom.h[1], prob.shape)
    iz, wz, dz = shape_weights_and_derivs((X[4] - geom.origin[2]) / geom.h[2], prob.shape)
    flat = (iz[:, None, None, :] * ny + iy[None, :, None, :]) * nx + ix[None, None, :, :]
    W = wz[:, None, None, :] * wy[None, :, None, :] * wx[None, None, :, :]
    gx = wz[:, None, None, :] * wy[None, :, None, :] * (dx[None, None, :, :] / geom.h[0])
    gy = wz[:, None, None, :] * (dy[None, :, None, :] / geom.h[1]) * wx[None, None, :, :]
    gz = (dz[:, None, None, :] / geom.h[2]) * wy[None, :, None, :] * wx[None, None, :, :]
    return flat, W, (gx, gy, gz)


# ----------------------------------------------------------------------------- transposes

def vector_deposit(A, X, geom, prob):
    """e_n = sum_i W(r_i - r_n) a_i for a (3, n) array A; result (3, nz, ny, nx)."""
    nx, ny, nz = prob.nodes
    flat, W, _ = _stencil_grad(X, geom, prob)
    out = np.empty((3, nz, ny, nx))
    for c in range(3):
        out[c] = np.bincount(flat.ravel(), weights=(W * A[c]).ravel(),
                             minlength=nx * ny * nz).reshape(nz, ny, nx)
    return out


def divergence_T(e, geom):
    """psi = -sum_c D_c^T e_c on nodes -1..n_a, shape (nz+2, ny+2, nx+2).

    (D_c phi)_n = (phi_{n+1} - phi_{n-1}) / (2 h_c) maps nodes -1..n_a to 0..n_a-1, so
    (D_c^T e)_m = (e_{m-1} - e_{m+1}) / (2 h_c) with e = 0 outside 0..n_a-1.
    """
    hx, hy, hz = geom.h_rest
    nz, ny, nx = e.shape[1:]
    psi = np.zeros((nz + 2, ny + 2, nx + 2))
    # -D^T e = (e_{m+1} - e_{m-1}) / (2h): e_n contributes +e_n/(2h) at m = n-1, -e_n/(2h) at m = n+1
    for c, h in ((0, hx), (1, hy), (2, hz)):
        ec = e[c] / (2.0 * h)
        sl_minus = [slice(1, -1)] * 3
        sl_plus = [slice(1, -1)] * 3
        ax = 2 - c  # array axis of component c (x is the last axis)
        sl_minus[ax] = slice(0, -2)   # m = n - 1
        sl_plus[ax] = slice(2, None)  # m = n + 1
        psi[tuple(sl_minus)] += ec
        psi[tuple(sl_plus)] -= ec
    return psi


def solve_ghost_source(psi, gbar):
    """chi_n = 1/(4 pi eps0) sum_m psi_m Gbar(n - m) for sources m on nodes -1..n_a and
    outputs n on nodes 0..n_a-1, by the zero-padded cyclic convolution with node -1 at
    index M-1 (every offset lies in [-n_a, n_a], which the Hockney array holds exactly)."""
    nz, ny, nx = (s - 2 for s in psi.shape)
    shape = (2 * nz, 2 * ny, 2 * nx)
    src = np.zeros(shape)
    idx = [np.concatenate([[m - 1], np.arange(n + 1)]) for m, n in zip(shape, (nz, ny, nx))]
    src[np.ix_(*idx)] = psi
    G = igf.hockney_array(gbar)
    axes = (0, 1, 2)
    conv = np.fft.irfftn(np.fft.rfftn(src, axes=axes) * np.fft.rfftn(G, axes=axes), s=shape,
                         axes=axes)
    return conv[:nz, :ny, :nx] / (4.0 * np.pi * EPS0)


def solve_field_T(e, kbars):
    """Transpose of pic.solve_field: with E'_a(n) = 1/(4 pi eps0) sum_m Kbar_a(n - m) Q_m and
    Kbar_a odd along a and even along the other axes, Qbar_m = sum_a sum_n Kbar_a(n - m) e_a(n)
    = -1/(4 pi eps0) sum_a (Kbar_a * e_a)(m), the same zero-padded convolutions (sources and
    outputs on nodes 0..n_a-1)."""
    return -sum(pic.solve_field(e[a], kbars)[a] for a in range(3))


def grad_gather(F, X, geom, prob):
    """sum_n grad W(r_i - r_n) F_n for a scalar grid F; result (3, n)."""
    flat, _, g = _stencil_grad(X, geom, prob)
    v = F.ravel()[flat]
    return np.stack([(gc * v).sum(axis=(0, 1, 2)) for gc in g])


def grad_gather_dot(E, A, X, geom, prob):
    """sum_n grad W(r_i - r_n) (a_i . E'_n) for the field E (3, nz, ny, nx); result (3, n)."""
    flat, _, g = _stencil_grad(X, geom, prob)
    s = sum(E[c].ravel()[flat] * A[c] for c in range(3))
    return np.stack([(gc * s).sum(axis=(0, 1, 2)) for gc in g])


def drift_T(lam, ell, prob):
    out = lam.copy()
    out[1] = lam[1] + ell * lam[0]
    out[3] = lam[3] + ell * lam[2]
    out[5] = lam[5] + ell * lam[4] / (prob.gamma * prob.gamma)
    return out


def quad_T(lam, K):
    out = lam.copy()
    out[0] = lam[0] - K * lam[1]
    out[2] = lam[2] + K * lam[3]
    return out


# ----------------------------------------------------------------------------- objective

def objective(X, w):
    _, _, m = pic.moments(X)
    return float(np.dot(w, m))


def objective_grad(X, w):
    """dJ/dX for J = w . (sigma_x, sigma_y, eps_x, eps_y)."""
    n = X.shape[1]
    mean, cov, m = pic.moments(X)
    D = X - mean[:, None]
    lam = np.zeros_like(X)
    sx, sy, ex, ey = m
    lam[0] += w[0] * D[0] / (n * sx)
    lam[2] += w[1] * D[2] / (n * sy)
    for (r, p, eps, wk) in ((0, 1, ex, w[2]), (2, 3, ey, w[3])):
        Sxx, Spp, Sxp = cov[r, r], cov[p, p], cov[r, p]
        lam[r] += wk * (Spp * D[r] - Sxp * D[p]) / (n * eps)
        lam[p] += wk * (Sxx * D[p] - Sxp * D[r]) / (n * eps)
    return lam


# ----------------------------------------------------------------------------- geometry

def geometry_adjoint(g, X2, geom, prob, e, E, Q, kernel):
    """(dJ/dmin (3,), dJ/dmax (3,)) of the box of the kick-point positions X2.

    g: (3, n) gradient of J with respect to the kick-point positions through the deposit's and
    the gather's weights at fixed geometry; e: dJ/dE' on the nodes (the vector deposit of the
    kick's adjoint); E: the step's E'; Q: its charge grid; kernel: Gbar (potential) or the
    three Kbar_a (direct field)."""
    nodes = np.asarray(prob.nodes, dtype=np.float64)
    h, o, hr = geom.h, geom.origin, geom.h_rest
    dJ_do = np.empty(3)
    dJ_dh = np.empty(3)
    for a, row in enumerate((0, 2, 4)):
        u = (X2[row] - o[a]) / h[a]
        dJ_do[a] = -np.sum(g[a])
        dJ_dh[a] = -np.sum(g[a] * u)
    nx, ny, nz = prob.nodes
    dJ_dhr = np.zeros(3)
    if prob.direct_field:
        for b in range(3):
            dK = [igf.field_cell_average_dh(nx, ny, nz, *hr, a, b) for a in range(3)]
            dE = pic.solve_field(Q, dK)
            dJ_dhr[b] = np.sum(e * dE)
    else:
        psi = divergence_T(e, geom)
        for b in range(3):
            dJ_dhr[b] = -np.sum(e[b] * E[b]) / hr[b]
            dG = igf.cell_average_dh(nx, ny, nz, *hr, b)
            dJ_dhr[b] += np.sum(Q * solve_ghost_source(psi, dG))
    dJ_dh += dJ_dhr * np.array([1.0, 1.0, prob.gamma])
    # h = (max - min)/(n - 3.5), origin = min - 1.25 h
    dJ_dmin = dJ_do * (1.0 + 1.25 / (nodes - 3.5)) - dJ_dh / (nodes - 3.5)
    dJ_dmax = -dJ_do * 1.25 / (nodes - 3.5) + dJ_dh / (nodes - 3.5)
    return dJ_dmin, dJ_dmax


def _kick_adjoint(lam, X2, geom, E, kernel, Q, ell, prob, follow_geometry):
    """lam at the kick point: adds the kick's position terms (direct, through the charge and,
    when the geometry follows the particles, through the box) to lam, which enters as the
    adjoint of the state after the kick."""
    A = np.stack([prob.C * ell * lam[1], prob.C * ell * lam[3],
                  prob.gamma * prob.C * ell * lam[5]])
    direct = grad_gather_dot(E, A, X2, geom, prob)
    e = vector_deposit(A, X2, geom, prob)
    chi = _charge_adjoint(e, geom, kernel, prob)
    g = direct + prob.q_macro * grad_gather(chi, X2, geom, prob)
    lam = lam.copy()
    for c, row in enumerate((0, 2, 4)):
        lam[row] = lam[row] + g[c]
    if follow_geometry:
        dmin, dmax = geometry_adjoint(g, X2, geom, prob, e, E, Q, kernel)
        for c, row in enumerate((0, 2, 4)):
            lam[row, np.argmin(X2[row])] += dmin[c]
            lam[row, np.argmax(X2[row])] += dmax[c]
    return lam


# ----------------------------------------------------------------------------- sweeps

def _green_and_field(Q, geom, prob):
    """The step's kernel(s) and E': the potential's Gbar and -grad phi, or (direct_field) the
    three field kernels and their convolutions."""
    if prob.direct_field:
        kbars = pic.green_field(geom, prob)
        return kbars, pic.solve_field(Q, kbars)
    gbar = pic.green(geom, prob)
    return gbar, pic.field(pic.solve(Q, gbar), geom)


def _charge_adjoint(e, geom, kernel, prob):
    """chi = dJ/dQ (per node) from the deposited adjoint field e: the transposed centred
    difference and the transposed (ghost-source) solve, or (direct_field) the transposed field
    convolutions."""
    if prob.direct_field:
        return solve_field_T(e, kernel)
    return solve_ghost_source(divergence_T(e, geom), kernel)


def forward(X0, ks, dss, n_steps, prob, geoms=None, space_charge=True):
    """Tracking as oracle.pic.track, optionally with frozen per-step geometries.  Returns the
    final state and, per step, (state at the step start, state at the kick point, geometry,
    E' grid, kernel, charge grid)."""
    rec = []
    X = X0
    n_el = len(ks)
    for j in range(n_steps):
        K, L = ks[j % n_el], dss[j % n_el]
        X1 = pic.thin_quad(X, K)
        X2 = pic.drift(X1, 0.5 * L, prob)
        if space_charge:
            geom = geoms[j] if geoms is not None else pic.geometry(X2, prob)
            Q = pic.deposit(X2, geom, prob)
            gbar, E = _green_and_field(Q, geom, prob)
            Ep = pic.gather(E, X2, geom, prob)
            X3 = pic.kick(X2, Ep, L, prob)
            rec.append((X, X2, geom, E, gbar, Q))
        else:
            X3 = X2
            rec.append((X, X2, None, None, None, None))
        X = pic.drift(X3, 0.5 * L, prob)
    return X, rec


def adjoint(X0, ks, dss, n_steps, prob, w, geoms=None, space_charge=True):
    """(J, dJ/dk (n_el,), dJ/dX0 (6, n), per-step geometries of the forward run)."""
    XN, rec = forward(X0, ks, dss, n_steps, prob, geoms, space_charge)
    lam = objective_grad(XN, w)
    n_el = len(ks)
    dk = np.zeros(n_el)
    for j in range(n_steps - 1, -1, -1):
        K, L = ks[j % n_el], dss[j % n_el]
        Xs, X2, geom, E, gbar, Q = rec[j]
        lam = drift_T(lam, 0.5 * L, prob)
        if space_charge:
            lam = _kick_adjoint(lam, X2, geom, E, gbar, Q, L, prob, geoms is None)
        lam = drift_T(lam, 0.5 * L, prob)
        dk[j % n_el] += float(np.sum(-Xs[0] * lam[1] + Xs[2] * lam[3]))
        lam = quad_T(lam, K)
    geoms_out = [r[2] for r in rec]
    return objective(XN, w), dk, lam, geoms_out


# ----------------------------------------------------------------------------- lattices of elements

def _half_T(lam, kind, k, ell, prob):
    """Transpose of half_map(., kind, k, ell) (drift, or the quadrupole matrix per plane with
    the longitudinal drift) applied to lam."""
    if kind != pic.QUAD:
        return drift_T(lam, 0.5 * ell, prob)
    Mx, My = pic.quad_matrix(k, 0.5 * ell), pic.quad_matrix(-k, 0.5 * ell)
    out = lam.copy()
    out[0] = Mx[0, 0] * lam[0] + Mx[1, 0] * lam[1]
    out[1] = Mx[0, 1] * lam[0] + Mx[1, 1] * lam[1]
    out[2] = My[0, 0] * lam[2] + My[1, 0] * lam[3]
    out[3] = My[0, 1] * lam[2] + My[1, 1] * lam[3]
    out[5] = lam[5] + 0.5 * ell * lam[4] / (prob.gamma * prob.gamma)
    return out


def _quad_dk(lam, X, k, ell):
    """sum over particles of lam . (d/dk of the half quadrupole map) X: the x plane sees
    quad_matrix(k), the y plane quad_matrix(-k), whose k-derivative is -quad_matrix_dk(-k)."""
    Dx = pic.quad_matrix_dk(k, 0.5 * ell)
    Dy = -pic.quad_matrix_dk(-k, 0.5 * ell)
    return float(np.sum(lam[0] * (Dx[0, 0] * X[0] + Dx[0, 1] * X[1]) +
                        lam[1] * (Dx[1, 0] * X[0] + Dx[1, 1] * X[1]) +
                        lam[2] * (Dy[0, 0] * X[2] + Dy[0, 1] * X[3]) +
                        lam[3] * (Dy[1, 0] * X[2] + Dy[1, 1] * X[3])))


def _slices_indexed(elements):
    """pic.slices with the index of the element each slice belongs to."""
    out = []
    for e, el in enumerate(elements):
        out.extend((kind, k, ell, e) for kind, k, ell in pic.slices([el]))
    return out


def forward_elements(X0, elements, n_steps, prob, geoms=None, space_charge=True):
    """Tracking as pic.track_elements (one slice per step, cycled), optionally with frozen
    per-step geometries.  Per step: (state at the start, after the first half map, after the
    kick, geometry, E' grid, kernel, charge grid)."""
    sl = _slices_indexed(elements)
    rec = []
    X = X0
    for j in range(n_steps):
        kind, k, ell, _ = sl[j % len(sl)]
        if kind == pic.THIN:
            X1 = pic.drift(pic.thin_quad(X, k), 0.5 * ell, prob)
        else:
            X1 = pic.half_map(X, kind, k, ell, prob)
        if space_charge:
            geom = geoms[j] if geoms is not None else pic.geometry(X1, prob)
            Q = pic.deposit(X1, geom, prob)
            gbar, E = _green_and_field(Q, geom, prob)
            X2 = pic.kick(X1, pic.gather(E, X1, geom, prob), ell, prob)
        else:
            geom = E = gbar = Q = None
            X2 = X1
        rec.append((X, X1, X2, geom, E, gbar, Q))
        X = pic.drift(X2, 0.5 * ell, prob) if kind == pic.THIN else \
            pic.half_map(X2, kind, k, ell, prob)
    return X, rec


def adjoint_elements(X0, elements, n_steps, prob, w, geoms=None, space_charge=True):
    """(J, dJ/dk per element (len(elements),), dJ/dX0, per-step geometries) for a lattice of
    (kind, k, ds, nslice) elements.  A quadrupole's strength enters both half maps of each of
    its slices: dJ/dk gets lam_after . (dM/dk) X_before for each.  A thin element's as in
    adjoint; drifts have no strength."""
    XN, rec = forward_elements(X0, elements, n_steps, prob, geoms, space_charge)
    lam = objective_grad(XN, w)
    sl = _slices_indexed(elements)
    dk = np.zeros(len(elements))
    for j in range(n_steps - 1, -1, -1):
        kind, k, ell, e = sl[j % len(sl)]
        Xs, X1, X2, geom, E, gbar, Q = rec[j]
        # second half map X2 -> X_{j+1}
        if kind == pic.QUAD:
            dk[e] += _quad_dk(lam, X2, k, ell)
        lam = _half_T(lam, kind, k, ell, prob)
        if space_charge:
            lam = _kick_adjoint(lam, X1, geom, E, gbar, Q, ell, prob, geoms is None)
        # first half map Xs -> X1
        if kind == pic.THIN:
            lam = drift_T(lam, 0.5 * ell, prob)
            dk[e] += float(np.sum(-Xs[0] * lam[1] + Xs[2] * lam[3]))
            lam = quad_T(lam, k)
        else:
            if kind == pic.QUAD:
                dk[e] += _quad_dk(lam, Xs, k, ell)
            lam = _half_T(lam, kind, k, ell, prob)
    return objective(XN, w), dk, lam, [r[3] for r in rec]


def cholesky_grad(L, xi, lamX0):
    """dJ/dSigma0 for X0 = L xi, L L^T = Sigma0, as the gradient with respect to the symmetric
    parameters (an off-diagonal pair Sigma_ab = Sigma_ba moves together): the Cholesky
    adjoint of Murray (2016), Sbar = L^-T Phi(L^T Lbar) L^-1, symmetrised, off-diagonal
    entries doubled."""
    Lbar = np.tril(lamX0 @ xi.T)
    P = L.T @ Lbar
    Phi = np.tril(P) - 0.5 * np.diag(np.diag(P))
    Linv = np.linalg.inv(L)
    S = Linv.T @ Phi @ Linv
    S = 0.5 * (S + S.T)
    G = 2.0 * S
    np.fill_diagonal(G, np.diag(S))
    return G
