"""Pins of the oracle's PIC step against closed forms, brute force and invariants."""
import numpy as np
import pytest
from scipy import integrate, special

import workloads
from oracle import igf, pic
from oracle.constants import C_LIGHT, E_CHARGE, EPS0

KE = 1.0 / (4.0 * np.pi * EPS0)


def _prob(nodes=(16, 16, 16), shape=1, n=1000, gamma_T=20.0):
    return pic.make_problem(n, -1.0e-6 / workloads.ELECTRON_MASS_MEV, 1e-9, gamma_T,
                            workloads.ELECTRON_MASS_MEV, nodes, shape)


def _beam(n, seed=0, sig=(1e-3, 1e-3, 2e-3)):
    r = np.random.default_rng(seed)
    X = np.zeros((6, n))
    X[0], X[2], X[4] = (r.standard_normal((3, n)) * np.array(sig)[:, None])
    X[1], X[3], X[5] = r.standard_normal((3, n)) * 1e-3
    return X


# ------------------------------------------------------------------ P1, P2: shapes, deposit

@pytest.mark.parametrize("shape", [1, 2])
def test_charge_conservation(shape):
    # the grid holds the configured bunch charge, 1 nC with the electron's sign (Listing 1's
    # add_particles(qm, charge_C, ...) takes the charge magnitude and the species' q/m); the
    # expected total is written from that configuration, not from the problem's macro charge
    prob = _prob(shape=shape, n=5000)
    X = _beam(5000)
    geom = pic.geometry(X, prob)
    Q = pic.deposit(X, geom, prob)
    assert abs(Q.sum() - (-1.0e-9)) < 1e-15 * 1.0e-9
    assert np.all(Q <= 0)  # electrons


@pytest.mark.parametrize("shape", [1, 2])
@pytest.mark.parametrize("n", [1, 7, 5000])
def test_one_particle_carries_the_bunch_charge_over_n(shape, n):
    # a single particle of an n-particle bunch deposits charge_C / n in total, spread by its
    # shape over 2^3 (CIC) or 3^3 (TSC) nodes; a wrong factor or a missing 1/n fails here
    prob = _prob(shape=shape, n=n)
    X = _beam(50, seed=9)
    geom = pic.geometry(X, prob)
    for i in (0, 17, 49):
        Q = pic.deposit(X[:, i:i + 1], geom, prob)
        assert abs(Q.sum() - (-1.0e-9 / n)) < 1e-15 * 1.0e-9 / n
        assert np.count_nonzero(Q) <= (shape + 1) ** 3


def test_shape_values_at_special_points():
    i, w = pic.shape_weights(np.array([3.0, 3.5]), 1)
    assert np.array_equal(i[:, 0], [3, 4]) and np.allclose(w[:, 0], [1.0, 0.0], atol=0)
    assert np.array_equal(i[:, 1], [3, 4]) and np.allclose(w[:, 1], [0.5, 0.5], atol=0)
    i, w = pic.shape_weights(np.array([3.0, 3.5]), 2)
    assert np.array_equal(i[:, 0], [2, 3, 4]) and np.array_equal(w[:, 0], [0.125, 0.75, 0.125])
    # a cell centre rounds up: d = -1/2 gives (1/2, 1/2, 0) on nodes (3, 4, 5)
    assert np.array_equal(i[:, 1], [3, 4, 5]) and np.array_equal(w[:, 1], [0.5, 0.5, 0.0])


@pytest.mark.parametrize("shape", [1, 2])
def test_shape_partition_of_unity_and_first_moment(shape):
    u = np.random.default_rng(1).uniform(2, 9, 1000)
    i, w = pic.shape_weights(u, shape)
    assert np.allclose(w.sum(axis=0), 1.0, atol=1e-15, rtol=0)
    assert np.allclose((w * (i - u)).sum(axis=0), 0.0, atol=1e-14)
    assert np.all(w >= 0)


def test_geometry_keeps_stencils_inside_and_rejects_degenerate_boxes():
    prob = _prob(nodes=(8, 9, 10), shape=2)
    X = _beam(1000, seed=4)
    geom = pic.geometry(X, prob)
    for ax, row in enumerate((0, 2, 4)):
        u = (X[row] - geom.origin[ax]) / geom.h[ax]
        assert abs(u.min() - 1.25) < 1e-12 and abs(u.max() - (prob.nodes[ax] - 2.25)) < 1e-12
    assert geom.h_rest[2] == prob.gamma * geom.h[2]
    X2 = X.copy()
    X2[2] = 0.0
    with pytest.raises(ValueError):
        pic.geometry(X2, prob)
    X2 = X.copy()
    X2[0, 5] = np.nan
    with pytest.raises(FloatingPointError):
        pic.geometry(X2, prob)


# ------------------------------------------------------------------ P5: Hockney = direct sum

@pytest.mark.parametrize("nodes,h", [((8, 8, 8), (1e-4, 1e-4, 3e-3)), ((5, 7, 6), (2e-4, 1e-4, 1e-4))])
def test_hockney_equals_direct_sum_including_ghost_nodes(nodes, h):
    nx, ny, nz = nodes
    rng = np.random.default_rng(7)
    Q = rng.standard_normal((nz, ny, nx)) * 1e-12
    g = igf.cell_average(nx, ny, nz, *h)
    phi = pic.solve(Q, g)
    # brute force: phi(n) = k sum_m Q_m Gbar(|n - m|) for n in -1..N
    ref = np.zeros_like(phi)
    for a in range(nz + 2):
        for b in range(ny + 2):
            for c in range(nx + 2):
                dz = np.abs(a - 1 - np.arange(nz))[:, None, None]
                dy = np.abs(b - 1 - np.arange(ny))[None, :, None]
                dx = np.abs(c - 1 - np.arange(nx))[None, None, :]
                ref[a, b, c] = KE * np.sum(Q * g[dz, dy, dx])
    assert np.abs(phi - ref).max() < 1e-13 * np.abs(ref).max()


# ------------------------------------------------------------------ P6: analytic Gaussian field

def _gauss_field(pts, sig, Q):
    """Rest-frame field of a 3-D Gaussian charge (textbook integral representation)."""
    out = np.zeros_like(pts)
    s2 = 2.0 * np.asarray(sig) ** 2
    for p in range(pts.shape[0]):
        x = pts[p]

        def f(u, c):
            t = np.exp(u)
            den = s2 + t
            val = np.exp(-np.sum(x ** 2 / den)) / np.sqrt(np.prod(den))
            return 2.0 * x[c] / den[c] * val * t

        for c in range(3):
            v, _ = integrate.quad(f, -40.0, 40.0, args=(c,), epsabs=0, epsrel=1e-12, limit=400)
            out[p, c] = KE * Q / np.sqrt(np.pi) * v
    return out


def test_integral_representation_matches_spherical_closed_form():
    sig = 1e-3
    Q = 1e-9
    pts = np.array([[0.5e-3, 0, 0], [0, 2e-3, 0], [1e-3, 1e-3, 1e-3]])
    E = _gauss_field(pts, (sig, sig, sig), Q)
    for p, e in zip(pts, E):
        r = np.linalg.norm(p)
        er = KE * Q / r ** 2 * (special.erf(r / (np.sqrt(2) * sig))
                                - np.sqrt(2 / np.pi) * r / sig * np.exp(-r ** 2 / (2 * sig ** 2)))
        assert np.allclose(e, er * p / r, rtol=1e-10, atol=0)


def _grid_field_of_gaussian(n, sig_lab, gamma, half=5.0, Q=1e-9):
    """E' from the oracle's solve and field for node-sampled Gaussian charge."""
    sig_lab = np.asarray(sig_lab)
    h = 2 * half * sig_lab / (n - 1)
    coords = [(np.arange(n) - (n - 1) / 2) * h[a] for a in range(3)]
    wts = [np.exp(-c ** 2 / (2 * s ** 2)) * hh / (np.sqrt(2 * np.pi) * s)
           for c, s, hh in zip(coords, sig_lab, h)]
    Qn = Q * wts[2][:, None, None] * wts[1][None, :, None] * wts[0][None, None, :]
    geom = pic.Geometry(np.array([c[0] for c in coords]), h,
                        np.array([h[0], h[1], gamma * h[2]]))
    g = igf.cell_average(n, n, n, *geom.h_rest)
    E = pic.field(pic.solve(Qn, g), geom)
    return E, coords, Qn.sum()


def test_field_of_round_gaussian_bunch_converges_at_second_order():
    gamma = 3.0
    sig_lab = (1e-3, 1e-3, 1.5e-3)
    sig_rest = (1e-3, 1e-3, gamma * 1.5e-3)
    errs = []
    for n in (17, 33):
        E, coords, Qtot = _grid_field_of_gaussian(n, sig_lab, gamma)
        c = (n - 1) // 2
        q = (n - 1) // 4
        idx = [(c + q, c, c), (c, c + q, c), (c, c, c + q), (c + q, c + q, c + q), (c - q, c, c + q // 2)]
        pts = np.array([[coords[0][i], coords[1][j], gamma * coords[2][k]] for (i, j, k) in idx])
        ref = _gauss_field(pts, sig_rest, Qtot)
        got = np.array([[E[a][k, j, i] for a in range(3)] for (i, j, k) in idx])
        errs.append(np.abs(got - ref).max() / np.abs(ref).max())
    assert errs[1] < 1e-2
    assert 3.5 < errs[0] / errs[1] < 4.5


# ------------------------------------------------------------------ P7, P8, P9: invariants

def _pic_field_at(X, prob, geom=None):
    geom = pic.geometry(X, prob) if geom is None else geom
    Q = pic.deposit(X, geom, prob)
    E = pic.field(pic.solve(Q, pic.green(geom, prob)), geom)
    return pic.gather(E, X, geom, prob)


@pytest.mark.parametrize("shape", [1, 2])
def test_momentum_conservation(shape):
    prob = _prob(nodes=(12, 10, 14), shape=shape, n=400)
    X = _beam(400, seed=5)
    Ep = _pic_field_at(X, prob)
    tot = np.abs(Ep).sum(axis=1)
    assert np.all(np.abs(Ep.sum(axis=1)) < 1e-13 * tot)
    X2 = _beam(2, seed=6)
    E2 = _pic_field_at(X2, prob)
    # equal and opposite, up to the FFT's rounding relative to the potential
    assert np.abs(E2[:, 0] + E2[:, 1]).max() < 1e-11 * np.abs(E2).max()


@pytest.mark.parametrize("shape", [1, 2])
def test_single_particle_on_a_node_feels_no_self_force(shape):
    prob = _prob(nodes=(9, 9, 9), shape=shape, n=1)
    geom = pic.Geometry(np.zeros(3), np.array([1e-4, 2e-4, 1e-4]),
                        np.array([1e-4, 2e-4, prob.gamma * 1e-4]))
    X = np.zeros((6, 1))
    X[0], X[2], X[4] = 4e-4, 8e-4, 4e-4  # node (4, 4, 4)
    E = _pic_field_at(X, prob, geom)
    Q = pic.deposit(X, geom, prob)
    scale = KE * abs(Q.sum()) / (1e-4) ** 2
    assert np.abs(E).max() < 1e-12 * scale


def test_direct_coulomb_sum_convergence():
    # three charges at least 8 cells apart: the PIC field converges to the Coulomb sum
    gamma_T = 0.5  # low energy so that the rest frame stays near-isotropic
    pos = np.array([[0.0, 0.0, 0.0], [3e-3, 1e-3, 0.5e-3], [-1e-3, 2.5e-3, 2e-3]])
    errs = []
    for n in (32, 64):
        prob = _prob(nodes=(n, n, n), shape=2, n=3, gamma_T=gamma_T)
        X = np.zeros((6, 3))
        X[0], X[2], X[4] = pos.T
        Ep = _pic_field_at(X, prob)
        rest = pos * np.array([1.0, 1.0, prob.gamma])
        ref = np.zeros((3, 3))
        for i in range(3):
            for j in range(3):
                if i != j:
                    d = rest[i] - rest[j]
                    ref[:, i] += KE * prob.q_macro * d / np.linalg.norm(d) ** 3
        errs.append(np.abs(Ep - ref).max() / np.abs(ref).max())
    assert errs[1] < 0.05
    assert errs[1] < errs[0]


@pytest.mark.parametrize("shape", [1, 2])
def test_mirror_symmetry(shape):
    prob = _prob(nodes=(12, 12, 12), shape=shape, n=300)
    X = _beam(300, seed=8)
    E = _pic_field_at(X, prob)
    for row, comp in ((0, 0), (2, 1), (4, 2)):
        Xm = X.copy()
        Xm[row] = -X[row]
        Em = _pic_field_at(Xm, prob)
        sign = np.ones(3)
        sign[comp] = -1.0
        assert np.abs(Em - sign[:, None] * E).max() < 1e-12 * np.abs(E).max()


# ------------------------------------------------------------------ P3: linear maps

def _matrix(f):
    M = np.zeros((6, 6))
    for c in range(6):
        e = np.zeros((6, 1))
        e[c] = 1.0
        M[:, c] = f(e)[:, 0]
    return M


def test_linear_maps_closed_form_and_symplectic():
    prob = _prob()
    g2 = prob.gamma ** 2
    D = _matrix(lambda X: pic.drift(X, 0.25, prob))
    ref = np.eye(6)
    ref[0, 1] = ref[2, 3] = 0.25
    ref[4, 5] = 0.25 / g2
    assert np.allclose(D, ref, rtol=1e-15, atol=0)
    Qm = _matrix(lambda X: pic.thin_quad(X, 1.3))
    ref = np.eye(6)
    ref[1, 0] = -1.3
    ref[3, 2] = 1.3
    assert np.array_equal(Qm, ref)
    J = np.kron(np.eye(3), np.array([[0.0, 1.0], [-1.0, 0.0]]))
    for M in (D, Qm):
        assert abs(np.linalg.det(M) - 1.0) < 1e-15
        assert np.allclose(M.T @ J @ M, J, atol=1e-15)


def test_thin_fodo_phase_advance_and_zero_current_tracking():
    prob = _prob()
    ks, dss = workloads.lattice_arrays(workloads.SMALL)
    cell = _matrix(lambda X: pic.track(X, ks, dss, 2, prob, space_charge=False))
    # textbook thin-lens FODO: cos mu = 1 - L^2 / (2 f^2) with f = 1 m, L = 0.5 m
    for b in (0, 2):
        mu = np.degrees(np.arccos(0.5 * np.trace(cell[b:b + 2, b:b + 2])))
        assert abs(mu - np.degrees(np.arccos(1.0 - 0.25 / 2.0))) < 1e-10
        assert abs(mu - 28.955) < 1e-3
    X0 = workloads.draw_xi(workloads.SMALL, n=2000) * 1e-3
    X = pic.track(X0, ks, dss, 20, prob, space_charge=False)
    M20 = np.linalg.matrix_power(cell, 10)
    assert np.abs(X - M20 @ X0).max() < 1e-15 * np.abs(X0).max() * 50
    _, _, m0 = pic.moments(X0)
    _, _, m1 = pic.moments(X)
    assert np.allclose(m1[2:], m0[2:], rtol=1e-12, atol=0)


# ------------------------------------------------------------------ kick constants from SI

def test_kick_constant_from_si_units():
    T, m = 20.0, workloads.ELECTRON_MASS_MEV
    prob = _prob(gamma_T=T)
    mass_kg = m * 1e6 * E_CHARGE / C_LIGHT ** 2
    gamma = (T + m) / m
    beta = np.sqrt(1.0 - 1.0 / gamma ** 2)
    p0 = gamma * mass_kg * beta * C_LIGHT
    q = -E_CHARGE
    Ep, L = 1.0, 1.0  # 1 V/m rest-frame field over 1 m
    dt = L / (beta * C_LIGHT)
    dpx = q * Ep / gamma * dt / p0          # lab transverse force q E'/gamma
    ddelta = q * Ep * dt / p0               # longitudinal force q E'_z
    assert abs(prob.C * Ep * L - dpx) < 1e-12 * abs(dpx)
    assert abs(prob.gamma * prob.C * Ep * L - ddelta) < 1e-12 * abs(ddelta)
    assert abs(prob.gamma - gamma) < 1e-14 * gamma


def test_space_charge_defocuses_a_round_beam():
    # repulsion: after a kick particles move outward in px, py
    prob = _prob(nodes=(16, 16, 16), shape=1, n=3000)
    X = _beam(3000, seed=9)
    X[[1, 3, 5]] = 0.0
    Y = pic.kick(X, pic.sc_field(X, prob), 0.5, prob)
    assert np.sum(Y[1] * X[0]) > 0 and np.sum(Y[3] * X[2]) > 0
