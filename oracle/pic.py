"""Space-charge PIC step in plain NumPy float64 (oracle; test infrastructure).

What the paper fixes (section "Model Assumptions"): s-based tracking by symplectic maps that
are linear about the reference orbit; one reference velocity for the whole bunch; space charge
electrostatic in the bunch rest frame, found by solving the Poisson equation there and applied
with a map-based split-operator.  It names the steps -- charge deposition, Poisson solve, beam
statistics (section "ImpactX") -- and the B-spline particle-shape order (Listing 1,
`set_particle_shape`).  The formulas below are readings where the paper is silent:

* Phase space (x, px, y, py, z, delta): x, y, z in m (z = lab longitudinal offset from the
  reference particle, head positive), px = p_x/p0, py = p_y/p0, delta = (p - p0)/p0.
* Reference particle from kinetic energy and rest mass: gamma = 1 + T/m.
* Macroparticle charge q_m = sign(q) Q/N.
* Grid: nx x ny x nz nodes (node-centred).  Each step the box is the particle min/max of
  x, y, z; h_a = (max_a - min_a)/(n_a - 3.5) and origin_a = min_a - 1.25 h_a.  The extreme
  particles then sit at u = 1.25 and u = n_a - 2.25, a quarter cell from the nearest node and
  from the nearest cell boundary, so every CIC and TSC stencil stays on nodes 0..n_a-1 and no
  particle of the box sits on a kink of either shape (where the tracked map would only have
  one-sided derivatives).  Rest frame: z' = gamma z, so the rest-frame cell is
  (hx, hy, gamma hz); node charges are frame-invariant.
* Shapes (B-spline order 1 and 2), u = (x - origin)/h:
  CIC  i = floor(u), f = u - i, weights (1-f, f) on nodes (i, i+1);
  TSC  i = floor(u + 1/2), d = u - i, weights (1/2 (1/2-d)^2, 3/4 - d^2, 1/2 (1/2+d)^2)
       on nodes (i-1, i, i+1); 3-D weights are tensor products.
* Poisson: phi_n = 1/(4 pi eps0) sum_m Q_m Gbar(n - m) with the integrated Green's function
  (oracle.igf), by Hockney's method: zero-pad to (2nz, 2ny, 2nx), cyclic convolution by FFT.
  phi is kept on nodes -1..n_a (the cyclic result is exact there).
* Field: E' = -grad phi by centred differences with spacings (hx, hy, gamma hz) on all nodes.
* Gather: the deposit's shape (momentum conserving).
* Kick over a length L (lab transverse force q E'/gamma, longitudinal q E'_z, divided by
  p0 beta c): dpx = C E'x L, dpy = C E'y L, ddelta = gamma C E'z L, C = (q/m)/(gamma^2 beta^2)
  with q/m in e/eV (the paper's qm_qeeV) and E' in V/m.
* Linear drift over l: x += l px, y += l py, z += l delta/gamma^2.
* Thin quadrupole of integrated strength K (1/m): px -= K x, py += K y.
* Step (split operator): thin quad K_j, drift L/2, space-charge kick over L with the field
  of the positions at that point, drift L/2.  The lattice (K_j, L_j) is cycled.
* Moments: centred second moments (1/N); geometric emittance
  eps_x = sqrt(<dx^2><dpx^2> - <dx dpx>^2) (unnormalised, as the paper quotes emittance).

Pins: tests/test_oracle_pic.py (charge conservation, shape values, Hockney vs direct
summation, analytic Gaussian-bunch field, direct Coulomb sums, momentum conservation, mirror
symmetry, closed-form maps and phase advance, kick constant from SI units),
tests/test_oracle_golden.py (the paper's printed emittance), tests/test_oracle_field.py (the
direct field, and the linear interior field of a uniformly charged ellipsoid) and
tests/test_oracle_envelope.py (multi-step tracking of a cold uniform ellipsoid against its
envelope equations).
"""
from dataclasses import dataclass

import numpy as np

from .constants import EPS0
from . import igf


@dataclass(frozen=True)
class Problem:
    """Constants of one beam: reference particle, species, grid, shape."""
    gamma: float
    gb2: float          # gamma^2 beta^2
    C: float            # kick constant (q/m)/(gamma^2 beta^2), 1/V
    q_macro: float      # charge per macroparticle, C
    nodes: tuple        # (nx, ny, nz)
    shape: int          # 1 = CIC, 2 = TSC
    direct_field: bool = False   # E' from the field's own IGF instead of -grad phi


def reference(kin_energy_MeV, mass_MeV):
    """gamma and gamma^2 beta^2 = (gamma-1)(gamma+1) of the reference particle."""
    t = kin_energy_MeV / mass_MeV
    gamma = 1.0 + t
    return gamma, t * (2.0 + t)


def make_problem(n, qm_qeeV, charge_C, kin_energy_MeV, mass_MeV, nodes, shape,
                 direct_field=False):
    gamma, gb2 = reference(kin_energy_MeV, mass_MeV)
    C = qm_qeeV / gb2
    q_macro = np.copysign(charge_C, qm_qeeV) / n
    return Problem(gamma, gb2, C, q_macro, tuple(int(v) for v in nodes), int(shape),
                   bool(direct_field))


def init_from_normals(sigma6, xi):
    """X = L xi with L the lower Cholesky factor of the 6x6 second-moment matrix."""
    L = np.linalg.cholesky(np.asarray(sigma6, dtype=np.float64))
    return L @ xi


# ----------------------------------------------------------------------------- geometry

@dataclass(frozen=True)
class Geometry:
    origin: np.ndarray   # (3,) lab origin of node 0, axes (x, y, z)
    h: np.ndarray        # (3,) lab spacings
    h_rest: np.ndarray   # (3,) rest-frame spacings (hx, hy, gamma hz)


def geometry(X, prob: Problem):
    pos = X[[0, 2, 4]]
    lo = pos.min(axis=1)
    hi = pos.max(axis=1)
    if not (np.all(np.isfinite(lo)) and np.all(np.isfinite(hi))):
        raise FloatingPointError("non-finite particle coordinate")
    ext = hi - lo
    if np.any(ext <= 0):
        raise ValueError("zero extent of the particle box")
    n = np.asarray(prob.nodes, dtype=np.float64)
    h = ext / (n - 3.5)
    origin = lo - 1.25 * h
    h_rest = np.array([h[0], h[1], prob.gamma * h[2]])
    return Geometry(origin, h, h_rest)


# ----------------------------------------------------------------------------- shapes

def shape_weights(u, shape):
    """Node indices and weights along one axis; returns (idx, w) of shape (S, n)."""
    if shape == 1:
        i = np.floor(u)
        f = u - i
        i = i.astype(np.int64)
        return np.stack([i, i + 1]), np.stack([1.0 - f, f])
    if shape == 2:
        i = np.floor(u + 0.5)
        d = u - i
        i = i.astype(np.int64)
        w = np.stack([0.5 * (0.5 - d) ** 2, 0.75 - d * d, 0.5 * (0.5 + d) ** 2])
        return np.stack([i - 1, i, i + 1]), w
    raise ValueError("shape must be 1 (CIC) or 2 (TSC)")


def _stencil(X, geom, prob):
    """Flattened node index and 3-D weight for every (particle, stencil point)."""
    nx, ny, nz = prob.nodes
    ix, wx = shape_weights((X[0] - geom.origin[0]) / geom.h[0], prob.shape)
    iy, wy = shape_weights((X[2] - geom.origin[1]) / geom.h[1], prob.shape)
    iz, wz = shape_weights((X[4] - geom.origin[2]) / geom.h[2], prob.shape)
    for a, na in ((ix, nx), (iy, ny), (iz, nz)):
        if a.min() < 0 or a.max() >= na:
            raise IndexError("stencil outside the grid")
    flat = (iz[:, None, None, :] * ny + iy[None, :, None, :]) * nx + ix[None, None, :, :]
    w = wz[:, None, None, :] * wy[None, :, None, :] * wx[None, None, :, :]
    return flat, w


def deposit(X, geom, prob: Problem):
    """Charge per node Q (coulomb), shape (nz, ny, nx)."""
    nx, ny, nz = prob.nodes
    flat, w = _stencil(X, geom, prob)
    Q = np.bincount(flat.ravel(), weights=(prob.q_macro * w).ravel(), minlength=nx * ny * nz)
    return Q.reshape(nz, ny, nx)


# ----------------------------------------------------------------------------- Poisson

def green(geom, prob: Problem):
    nx, ny, nz = prob.nodes
    hx, hy, hz = geom.h_rest
    return igf.cell_average(nx, ny, nz, hx, hy, hz)


def solve(Q, gbar):
    """phi on nodes -1..n_a (shape (nz+2, ny+2, nx+2)) by zero-padded FFT convolution."""
    nz, ny, nx = Q.shape
    shape = (2 * nz, 2 * ny, 2 * nx)
    Gfull = igf.hockney_array(gbar)
    Qpad = np.zeros(shape)
    Qpad[:nz, :ny, :nx] = Q
    axes = (0, 1, 2)
    conv = np.fft.irfftn(np.fft.rfftn(Qpad, axes=axes) * np.fft.rfftn(Gfull, axes=axes),
                         s=shape, axes=axes)
    keep = [np.concatenate([[m - 1], np.arange(n + 1)]) for m, n in zip(shape, (nz, ny, nx))]
    return conv[np.ix_(*keep)] / (4.0 * np.pi * EPS0)


def field(phi, geom):
    """Rest-frame E' = -grad phi on nodes 0..n_a-1, shape (3, nz, ny, nx), rows (x, y, z)."""
    hx, hy, hz = geom.h_rest
    Ex = -(phi[1:-1, 1:-1, 2:] - phi[1:-1, 1:-1, :-2]) / (2.0 * hx)
    Ey = -(phi[1:-1, 2:, 1:-1] - phi[1:-1, :-2, 1:-1]) / (2.0 * hy)
    Ez = -(phi[2:, 1:-1, 1:-1] - phi[:-2, 1:-1, 1:-1]) / (2.0 * hz)
    return np.stack([Ex, Ey, Ez])


def green_field(geom, prob: Problem):
    """The three field kernels Kbar_x, Kbar_y, Kbar_z on the octant (igf.field_cell_average)."""
    nx, ny, nz = prob.nodes
    hx, hy, hz = geom.h_rest
    return [igf.field_cell_average(nx, ny, nz, hx, hy, hz, a) for a in range(3)]


def solve_field(Q, kbars):
    """Rest-frame E' on nodes 0..n_a-1, shape (3, nz, ny, nx): the charge of every cell taken
    as spread uniformly over the cell (the IGF reading), E'_a(n) = 1/(4 pi eps0)
    sum_m Q_m Kbar_a(n - m), by the same zero-padded FFT convolution as solve (reading 20)."""
    nz, ny, nx = Q.shape
    shape = (2 * nz, 2 * ny, 2 * nx)
    Qpad = np.zeros(shape)
    Qpad[:nz, :ny, :nx] = Q
    axes = (0, 1, 2)
    Qh = np.fft.rfftn(Qpad, axes=axes)
    out = []
    for a in range(3):
        K = igf.hockney_array_field(kbars[a], a)
        conv = np.fft.irfftn(Qh * np.fft.rfftn(K, axes=axes), s=shape, axes=axes)
        out.append(conv[:nz, :ny, :nx] / (4.0 * np.pi * EPS0))
    return np.stack(out)


def gather(E, X, geom, prob: Problem):
    """Field at the particles, shape (3, n)."""
    flat, w = _stencil(X, geom, prob)
    out = np.empty((3, X.shape[1]))
    for c in range(3):
        out[c] = (E[c].ravel()[flat] * w).sum(axis=(0, 1, 2))
    return out


def sc_field(X, prob: Problem):
    """Geometry, deposit, IGF, Poisson solve, field and gather for the positions in X."""
    geom = geometry(X, prob)
    Q = deposit(X, geom, prob)
    if prob.direct_field:
        E = solve_field(Q, green_field(geom, prob))
    else:
        E = field(solve(Q, green(geom, prob)), geom)
    return gather(E, X, geom, prob)


# ----------------------------------------------------------------------------- maps

def drift(X, ell, prob: Problem):
    Y = X.copy()
    Y[0] = X[0] + ell * X[1]
    Y[2] = X[2] + ell * X[3]
    Y[4] = X[4] + ell * X[5] / (prob.gamma * prob.gamma)
    return Y


def thin_quad(X, K):
    Y = X.copy()
    Y[1] = X[1] - K * X[0]
    Y[3] = X[3] + K * X[2]
    return Y


def kick(X, Ep, L, prob: Problem):
    Y = X.copy()
    Y[1] = X[1] + prob.C * Ep[0] * L
    Y[3] = X[3] + prob.C * Ep[1] * L
    Y[5] = X[5] + prob.gamma * prob.C * Ep[2] * L
    return Y


def step(X, K, L, prob: Problem, space_charge=True):
    X = thin_quad(X, K)
    X = drift(X, 0.5 * L, prob)
    if space_charge:
        X = kick(X, sc_field(X, prob), L, prob)
    return drift(X, 0.5 * L, prob)


def track(X, ks, dss, n_steps, prob: Problem, space_charge=True):
    """Apply n_steps steps; step j uses (ks[j mod n_el], dss[j mod n_el])."""
    n_el = len(ks)
    for j in range(n_steps):
        X = step(X, ks[j % n_el], dss[j % n_el], prob, space_charge)
    return X


# ----------------------------------------------------------------------------- thick elements
# Listing 1 of the paper builds its FODO from Drift(ds, nslice) and Quad(ds, k, nslice); with
# space charge each element is cut into nslice slices, and each slice is the split-operator
# step of section "Model Assumptions": the element's linear map over half the slice, the
# space-charge kick over the slice, the map over the other half.  Element kinds:
THIN, DRIFT, QUAD = 0, 1, 2   # THIN: thin quad k then the space-charge drift ds (one slice)


def quad_matrix(k, s):
    """(x, px) transfer matrix of a quadrupole of strength k [1/m^2] over length s, focusing
    for k > 0 (x'' = -k x): [[cos p, sin p / sqrt k], [-sqrt k sin p, cos p]], p = sqrt(k) s;
    cosh / sinh for k < 0; a drift for k = 0.  The y plane sees -k."""
    if k > 0:
        r = np.sqrt(k)
        c, sn = np.cos(r * s), np.sin(r * s)
        return np.array([[c, sn / r], [-r * sn, c]])
    if k < 0:
        r = np.sqrt(-k)
        c, sn = np.cosh(r * s), np.sinh(r * s)
        return np.array([[c, sn / r], [r * sn, c]])
    return np.array([[1.0, s], [0.0, 1.0]])


def quad_matrix_dk(k, s):
    """Derivative with respect to k of quad_matrix(k, s), entry by entry: from the closed forms
    (d/dk cos(sqrt(k) s) = -s sin(sqrt(k) s) / (2 sqrt k), ...) for |k| s^2 >= 0.1, else from
    the power series in k of cos(sqrt(k) s), sin(sqrt(k) s)/sqrt(k) and -sqrt(k) sin(sqrt(k) s),
    which hold for either sign of k (the closed forms cancel badly near k = 0)."""
    if abs(k) * s * s >= 0.1:
        if k > 0:
            r = np.sqrt(k)
            c, sn = np.cos(r * s), np.sin(r * s)
            dc = -s * sn / (2.0 * r)
            return np.array([[dc, s * c / (2.0 * k) - sn / (2.0 * r ** 3)],
                             [-sn / (2.0 * r) - 0.5 * s * c, dc]])
        r = np.sqrt(-k)
        c, sn = np.cosh(r * s), np.sinh(r * s)
        dc = -s * sn / (2.0 * r)
        return np.array([[dc, s * c / (2.0 * k) + sn / (2.0 * r ** 3)],
                         [-sn / (2.0 * r) - 0.5 * s * c, dc]])
    # cos = sum_m (-k)^m s^2m/(2m)!, sin/sqrt(k) = sum_m (-k)^m s^(2m+1)/(2m+1)!,
    # -sqrt(k) sin = -sum_m (-1)^m k^(m+1) s^(2m+1)/(2m+1)!: differentiate term by term
    d00 = d01 = d10 = 0.0
    fact = [1.0]
    for q in range(1, 40):
        fact.append(fact[-1] * q)
    for m in range(1, 16):
        d00 += m * (-1) ** m * k ** (m - 1) * s ** (2 * m) / fact[2 * m]
        d01 += m * (-1) ** m * k ** (m - 1) * s ** (2 * m + 1) / fact[2 * m + 1]
    for m in range(0, 16):
        d10 -= (m + 1) * (-1) ** m * k ** m * s ** (2 * m + 1) / fact[2 * m + 1]
    return np.array([[d00, d01], [d10, d00]])


def thick_quad(X, k, s, prob: Problem):
    """Quadrupole map over length s; the longitudinal plane drifts (z += s delta / gamma^2)."""
    Mx, My = quad_matrix(k, s), quad_matrix(-k, s)
    Y = X.copy()
    Y[0] = Mx[0, 0] * X[0] + Mx[0, 1] * X[1]
    Y[1] = Mx[1, 0] * X[0] + Mx[1, 1] * X[1]
    Y[2] = My[0, 0] * X[2] + My[0, 1] * X[3]
    Y[3] = My[1, 0] * X[2] + My[1, 1] * X[3]
    Y[4] = X[4] + s * X[5] / (prob.gamma * prob.gamma)
    return Y


def slices(elements):
    """Expand (kind, k, ds, nslice) elements into the per-step list (kind, k, slice length)."""
    out = []
    for kind, k, ds, ns in elements:
        ns = max(int(ns), 1) if kind != THIN else 1
        out.extend([(kind, k, ds / ns)] * ns)
    return out


def half_map(X, kind, k, ell, prob: Problem):
    """The linear map of half a slice of length ell (a thin slice's first half applies its quad
    first; its second half is the plain drift, see slice_step)."""
    if kind == QUAD:
        return thick_quad(X, k, 0.5 * ell, prob)
    return drift(X, 0.5 * ell, prob)


def slice_step(X, kind, k, ell, prob: Problem, space_charge=True):
    if kind == THIN:
        return step(X, k, ell, prob, space_charge)
    X = half_map(X, kind, k, ell, prob)
    if space_charge:
        X = kick(X, sc_field(X, prob), ell, prob)
    return half_map(X, kind, k, ell, prob)


def track_elements(X, elements, n_steps, prob: Problem, space_charge=True):
    """n_steps slices through the lattice (kind, k, ds, nslice), cycled."""
    sl = slices(elements)
    for j in range(n_steps):
        kind, k, ell = sl[j % len(sl)]
        X = slice_step(X, kind, k, ell, prob, space_charge)
    return X


# ----------------------------------------------------------------------------- distributions

def sigma_from_params(sigmaX, sigmaY, sigmaT, sigmaPx, sigmaPy, sigmaPt, muxpx, muypy, mutpt):
    """6x6 covariance (x, px, y, py, z, delta) of the distribution parameters of Listing 1
    (`distribution.Waterbag(sigmaX, ..., muxpx, muypy, mutpt)`).  Reading (the paper prints the
    parameters, not their definition): in each plane (u, pu) the rms size is
    sigmaU / sqrt(1 - muupu^2), the rms momentum sigmaPu / sqrt(1 - muupu^2) and the correlation
    coefficient -muupu; the Listing's (t, pt) pair is taken as (z, delta)."""
    S = np.zeros((6, 6))
    for i, (su, sp, mu) in enumerate(((sigmaX, sigmaPx, muxpx), (sigmaY, sigmaPy, muypy),
                                      (sigmaT, sigmaPt, mutpt))):
        if not (su > 0 and sp > 0 and abs(mu) < 1):
            raise ValueError("sigmas must be positive and |mu| < 1")
        c = 1.0 / np.sqrt(1.0 - mu * mu)
        ru, rp = su * c, sp * c
        S[2 * i, 2 * i] = ru * ru
        S[2 * i + 1, 2 * i + 1] = rp * rp
        S[2 * i, 2 * i + 1] = S[2 * i + 1, 2 * i] = -mu * ru * rp
    return S


WATERBAG_RADIUS = np.sqrt(8.0)   # a uniform 6-ball of this radius has unit covariance


def init_waterbag(sigma6, xi_ball):
    """Waterbag beam: uniform density inside the 6-D ellipsoid x^T Sigma^-1 x <= 8, whose
    covariance is Sigma (reading: the paper names the distribution only).  xi_ball (6, n) are
    points uniform in the ball of radius sqrt(8) (unit covariance); x = L xi with L the lower
    Cholesky factor of Sigma, as for the Gaussian beam."""
    return init_from_normals(sigma6, xi_ball)


# ----------------------------------------------------------------------------- statistics

def moments(X):
    """Mean (6,), centred covariance (6, 6) and (sigma_x, sigma_y, eps_x, eps_y)."""
    mean = X.mean(axis=1)
    D = X - mean[:, None]
    cov = (D @ D.T) / X.shape[1]
    sx = np.sqrt(cov[0, 0])
    sy = np.sqrt(cov[2, 2])
    ex = np.sqrt(cov[0, 0] * cov[1, 1] - cov[0, 1] ** 2)
    ey = np.sqrt(cov[2, 2] * cov[3, 3] - cov[2, 3] ** 2)
    return mean, cov, np.array([sx, sy, ex, ey])
