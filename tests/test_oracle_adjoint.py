"""Pins of the oracle's reverse sweep: dot-product tests of each transposed operation, central
finite differences with space charge (of the tracking, whose grid geometry follows the
particles, and of the same map with the geometry frozen), the kernels' h-derivatives, and the
closed-form gradient of the zero-current map."""
import numpy as np
import pytest

import workloads
from oracle import adjoint as adj
from oracle import igf, pic

W4 = np.array([0.7, -0.4, 1.3, 0.9])   # weights on (sigma_x, sigma_y, eps_x, eps_y)


def _prob(nodes=(12, 12, 12), shape=1, n=400):
    c = workloads.SMALL
    return pic.make_problem(n, c.qm_qeeV, c.charge_C, c.kin_energy_MeV, c.mass_MeV, nodes, shape)


def _beam(n, seed=0):
    r = np.random.default_rng(seed)
    X = np.zeros((6, n))
    X[0], X[2], X[4] = r.standard_normal((3, n)) * np.array([1e-3, 1e-3, 2e-3])[:, None]
    X[1], X[3], X[5] = r.standard_normal((3, n)) * 1e-3
    return X


@pytest.mark.parametrize("shape", [1, 2])
def test_transposes_by_dot_products(shape):
    prob = _prob(nodes=(10, 9, 12), shape=shape, n=300)
    X = _beam(300, seed=1)
    geom = pic.geometry(X, prob)
    r = np.random.default_rng(2)
    nx, ny, nz = prob.nodes
    # vector deposit is the transpose of the gather
    A = r.standard_normal((3, 300))
    F = r.standard_normal((3, nz, ny, nx))
    lhs = np.sum(adj.vector_deposit(A, X, geom, prob) * F)
    rhs = np.sum(A * pic.gather(F, X, geom, prob))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    # -D^T is the transpose of the field operator E' = -D phi
    e = r.standard_normal((3, nz, ny, nx))
    phi = r.standard_normal((nz + 2, ny + 2, nx + 2))
    lhs = np.sum(adj.divergence_T(e, geom) * phi)
    rhs = np.sum(e * pic.field(phi, geom))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    # the ghost-source convolution is the transpose of the solve (Gbar is even)
    gbar = pic.green(geom, prob)
    psi = r.standard_normal((nz + 2, ny + 2, nx + 2))
    rho = r.standard_normal((nz, ny, nx))
    lhs = np.sum(adj.solve_ghost_source(psi, gbar) * rho)
    rhs = np.sum(psi * pic.solve(rho, gbar))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


@pytest.mark.parametrize("shape", [1, 2])
def test_grad_gather_is_the_position_derivative_of_the_deposit(shape):
    prob = _prob(nodes=(10, 10, 10), shape=shape, n=50)
    X = _beam(50, seed=3)
    geom = pic.geometry(X, prob)
    F = np.random.default_rng(4).standard_normal((10, 10, 10))
    g = prob.q_macro * adj.grad_gather(F, X, geom, prob)
    for i in (0, 17, 42):
        for c, row in enumerate((0, 2, 4)):
            h = 1e-7 * geom.h[c]
            Xp, Xm = X.copy(), X.copy()
            Xp[row, i] += h
            Xm[row, i] -= h
            fd = (np.sum(pic.deposit(Xp, geom, prob) * F)
                  - np.sum(pic.deposit(Xm, geom, prob) * F)) / (2 * h)
            assert abs(fd - g[c, i]) < 1e-6 * np.abs(g).max()


def _fd(fun, x0, h):
    return (fun(x0 + h) - fun(x0 - h)) / (2 * h)


def _frozen(X0, ks, dss, steps, prob):
    """The per-step geometries of the forward run, to freeze them."""
    return [r[2] for r in adj.forward(X0, ks, dss, steps, prob)[1]]


# bars of the central-difference checks (step 1e-6 relative): measured 3e-11 .. 2e-10 for dJ/dk
# and 8e-10 .. 3.5e-9 for directional derivatives in X0 with the geometry following the
# particles; the frozen-geometry checks keep 1e-6
FD_BARS = {True: (1e-8, 1e-7), False: (1e-6, 1e-6)}
# relative rounding noise of a computed objective after a few steps with FFT solves: a central
# difference with step t then carries up to J_NOISE |J| / t, which matters where the
# directional derivative is small against J / t
J_NOISE = 1e-14


@pytest.mark.parametrize("follow", [True, False])
@pytest.mark.parametrize("shape", [1, 2])
def test_adjoint_matches_central_differences_with_space_charge(shape, follow):
    # follow=True: the tracking itself, whose grid geometry follows the particles' box every
    # step; follow=False: the same map with every step's geometry frozen to the forward run's
    n, steps = 400, 4
    prob = _prob(nodes=(12, 12, 12), shape=shape, n=n)
    X0 = _beam(n, seed=5)
    ks = np.array([1.0, -1.0, 0.8])
    dss = np.array([0.5, 0.5, 0.5])
    geoms = None if follow else _frozen(X0, ks, dss, steps, prob)
    J, dk, lam0, _ = adj.adjoint(X0, ks, dss, steps, prob, W4, geoms=geoms)

    def J_of(ks_, X_=X0):
        if follow:
            return adj.objective(pic.track(X_, ks_, dss, steps, prob), W4)
        XN, _ = adj.forward(X_, ks_, dss, steps, prob, geoms=geoms)
        return adj.objective(XN, W4)

    bar_k, bar_x = FD_BARS[follow]
    assert abs(J_of(ks) - J) < 1e-15 * abs(J)
    for j in range(3):
        h = 1e-6 * abs(ks[j])
        e = np.zeros(3)
        e[j] = 1.0
        fd = _fd(lambda t: J_of(ks + t * e), 0.0, h)
        assert abs(fd - dk[j]) < bar_k * np.abs(dk).max()
    # directional derivative along a random perturbation of X0
    D = np.random.default_rng(6).standard_normal(X0.shape) * X0.std(axis=1)[:, None]
    fd = _fd(lambda t: J_of(ks, X0 + t * D), 0.0, 1e-6)
    assert abs(fd - np.sum(lam0 * D)) < bar_x * abs(np.sum(lam0 * D)) + J_NOISE * abs(J) / 1e-6


@pytest.mark.parametrize("direct", [False, True])
def test_geometry_terms_are_a_measurable_part_of_the_gradient(direct):
    # the box terms change dJ/dk by 1e-4 .. 1e-3 of its largest entry on this beam, far above
    # the 1e-8 bar of the central-difference check, so that check sees a missing or wrong term
    n, steps = 400, 4
    c = workloads.SMALL
    prob = pic.make_problem(n, c.qm_qeeV, c.charge_C, c.kin_energy_MeV, c.mass_MeV,
                            (12, 12, 12), 1, direct_field=direct)
    X0 = _beam(n, seed=5)
    ks = np.array([1.0, -1.0, 0.8])
    dss = np.array([0.5, 0.5, 0.5])
    _, dk, _, _ = adj.adjoint(X0, ks, dss, steps, prob, W4)
    _, dkf, _, _ = adj.adjoint(X0, ks, dss, steps, prob, W4,
                               geoms=_frozen(X0, ks, dss, steps, prob))
    assert np.abs(dk - dkf).max() > 1e-5 * np.abs(dk).max()


def test_kernel_h_derivatives():
    # dGbar/dh_b and dKbar_a/dh_b of the anisotropic rest-frame cell against central
    # differences of the kernels (step 1e-5 h_b, truncation ~1e-10) and Euler's identity for
    # homogeneous functions: Gbar has degree -1 in h, Kbar_a degree -2
    nx, ny, nz = 6, 5, 7
    h = np.array([1.3e-4, 0.9e-4, 4.1e-3])
    G = igf.cell_average(nx, ny, nz, *h)
    dG = [igf.cell_average_dh(nx, ny, nz, *h, b) for b in range(3)]
    assert np.abs(sum(h[b] * dG[b] for b in range(3)) + G).max() < 1e-14 * np.abs(G).max()

    def fd(f, b):
        hp, hm = h.copy(), h.copy()
        hp[b] += 1e-5 * h[b]
        hm[b] -= 1e-5 * h[b]
        return (f(hp) - f(hm)) / (2e-5 * h[b])

    for b in range(3):
        d = fd(lambda hh: igf.cell_average(nx, ny, nz, *hh), b)
        assert np.abs(d - dG[b]).max() < 1e-8 * np.abs(dG[b]).max()
    for a in range(3):
        K = igf.field_cell_average(nx, ny, nz, *h, a)
        dK = [igf.field_cell_average_dh(nx, ny, nz, *h, a, b) for b in range(3)]
        assert np.abs(sum(h[b] * dK[b] for b in range(3)) + 2 * K).max() < \
            1e-14 * np.abs(K).max()
        for b in range(3):
            d = fd(lambda hh: igf.field_cell_average(nx, ny, nz, *hh, a), b)
            assert np.abs(d - dK[b]).max() < 1e-8 * np.abs(dK[b]).max()


def _matrix(f):
    M = np.zeros((6, 6))
    for c in range(6):
        e = np.zeros((6, 1))
        e[c] = 1.0
        M[:, c] = f(e)[:, 0]
    return M


def test_zero_current_gradient_in_closed_form():
    # without space charge the map is linear, X_N = M X0 with M a product of drift and thin-quad
    # matrices; dM/dk_e is the sum over the steps that use element e of (after) D dQ (before)
    n, steps = 500, 7
    prob = _prob(n=n)
    X0 = _beam(n, seed=7)
    ks = np.array([1.1, -0.9, 0.7])
    dss = np.array([0.5, 0.4, 0.6])
    J, dk, lam0, _ = adj.adjoint(X0, ks, dss, steps, prob, W4, space_charge=False)
    Ps = [_matrix(lambda X, j=j: pic.drift(pic.drift(pic.thin_quad(X, ks[j % 3]),
                                                     0.5 * dss[j % 3], prob),
                                            0.5 * dss[j % 3], prob)) for j in range(steps)]
    M = np.eye(6)
    for P in Ps:
        M = P @ M
    XN = M @ X0
    Lam = adj.objective_grad(XN, W4)
    assert np.allclose(lam0, M.T @ Lam, rtol=1e-12, atol=1e-12 * np.abs(lam0).max())
    dQ = np.zeros((6, 6))
    dQ[1, 0], dQ[3, 2] = -1.0, 1.0
    for e in range(3):
        dM = np.zeros((6, 6))
        for s in range(steps):
            if s % 3 != e:
                continue
            before = np.eye(6)
            for P in Ps[:s]:
                before = P @ before
            after = np.eye(6)
            for P in Ps[s + 1:]:
                after = P @ after
            Dfull = _matrix(lambda X: pic.drift(pic.drift(X, 0.5 * dss[e], prob), 0.5 * dss[e], prob))
            dM += after @ Dfull @ dQ @ before
        ref = np.sum(Lam * (dM @ X0))
        assert abs(dk[e] - ref) < 1e-12 * np.abs(dk).max()


def test_sigma0_gradient_through_the_cholesky_factor():
    n, steps = 300, 3
    prob = _prob(nodes=(10, 10, 10), shape=2, n=n)
    xi = np.random.default_rng(8).standard_normal((6, n))
    S0 = np.diag(np.array([1e-3, 1e-3, 1.2e-3, 0.9e-3, 2e-3, 1e-3]) ** 2)
    S0[0, 1] = S0[1, 0] = 0.3e-6
    S0[2, 4] = S0[4, 2] = -0.5e-6
    ks = np.array([1.0, -1.0])
    dss = np.array([0.5, 0.5])
    L = np.linalg.cholesky(S0)
    J, dk, lam0, _ = adj.adjoint(L @ xi, ks, dss, steps, prob, W4)
    G = adj.cholesky_grad(L, xi, lam0)

    def J_of(S):
        return adj.objective(pic.track(np.linalg.cholesky(S) @ xi, ks, dss, steps, prob), W4)

    for (a, b) in ((0, 0), (0, 1), (2, 4), (3, 3), (1, 5)):
        h = 1e-6 * np.sqrt(S0[a, a] * S0[b, b])
        E = np.zeros((6, 6))
        E[a, b] = E[b, a] = 1.0
        fd = (J_of(S0 + h * E) - J_of(S0 - h * E)) / (2 * h)
        assert abs(fd - G[a, b]) < 1e-5 * np.abs(G).max()


@pytest.mark.parametrize("k", [1.3, -0.7, 0.02, -1e-9, 0.0])
def test_quad_matrix_k_derivative(k):
    # against central differences of the matrix itself (series branch for |k| s^2 < 0.1)
    s = 0.45
    D = pic.quad_matrix_dk(k, s)
    h = 1e-5
    fd = (pic.quad_matrix(k + h, s) - pic.quad_matrix(k - h, s)) / (2 * h) if k != 0.0 else \
        (pic.quad_matrix(h, s) - pic.quad_matrix(-h, s)) / (2 * h)
    assert np.abs(D - fd).max() < 1e-8
    if k == 0.0:   # the limit of the closed forms: [[-s^2/2, -s^3/6], [-s, -s^2/2]]
        assert np.allclose(D, [[-s * s / 2, -s ** 3 / 6], [-s, -s * s / 2]], rtol=1e-15, atol=0)
    # the two branches meet at |k| s^2 = 0.1
    kb = 0.1 / (s * s)
    for sg in (1, -1):
        a = pic.quad_matrix_dk(sg * kb * (1 + 1e-12), s)
        b = pic.quad_matrix_dk(sg * kb * (1 - 1e-12), s)
        assert np.abs(a - b).max() < 1e-12 * np.abs(a).max()


THICK = [(pic.DRIFT, 0.0, 0.3, 2), (pic.QUAD, 1.4, 0.6, 3), (pic.THIN, -0.6, 0.4, 1),
         (pic.QUAD, -1.1, 0.5, 2)]


def _frozen_elements(X0, els, steps, prob):
    return [r[3] for r in adj.forward_elements(X0, els, steps, prob)[1]]


@pytest.mark.parametrize("follow", [True, False])
@pytest.mark.parametrize("shape", [1, 2])
def test_thick_lattice_adjoint_matches_central_differences(shape, follow):
    n, steps = 300, 9
    prob = _prob(nodes=(12, 10, 12), shape=shape, n=n)
    X0 = _beam(n, seed=9)
    geoms = None if follow else _frozen_elements(X0, THICK, steps, prob)
    J, dk, lam0, _ = adj.adjoint_elements(X0, THICK, steps, prob, W4, geoms=geoms)

    def J_of(els, X_=X0):
        XN, _ = adj.forward_elements(X_, els, steps, prob, geoms=geoms)
        return adj.objective(XN, W4)

    bar_k, bar_x = FD_BARS[follow]

    assert abs(J_of(THICK) - J) < 1e-15 * abs(J)
    # the same tracking as pic.track_elements when the geometry is not frozen
    XN, _ = adj.forward_elements(X0, THICK, steps, prob)
    assert np.array_equal(XN, pic.track_elements(X0, THICK, steps, prob))
    assert dk[0] == 0.0                      # a drift has no strength
    for e in (1, 2, 3):
        h = 1e-6 * abs(THICK[e][1])

        def shifted(t, e=e):
            els = list(THICK)
            kind, k, ds, ns = els[e]
            els[e] = (kind, k + t, ds, ns)
            return J_of(els)

        fd = _fd(shifted, 0.0, h)
        assert abs(fd - dk[e]) < bar_k * np.abs(dk).max(), e
    D = np.random.default_rng(10).standard_normal(X0.shape) * X0.std(axis=1)[:, None]
    fd = _fd(lambda t: J_of(THICK, X0 + t * D), 0.0, 1e-6)
    assert abs(fd - np.sum(lam0 * D)) < bar_x * abs(np.sum(lam0 * D)) + J_NOISE * abs(J) / 1e-6


def test_thin_elements_reduce_to_the_thin_sweep():
    n, steps = 250, 5
    prob = _prob(n=n)
    X0 = _beam(n, seed=11)
    ks = np.array([1.0, -0.8])
    dss = np.array([0.5, 0.4])
    J, dk, lam0, _ = adj.adjoint(X0, ks, dss, steps, prob, W4)
    J2, dk2, lam2, _ = adj.adjoint_elements(X0, [(pic.THIN, k, d, 1) for k, d in zip(ks, dss)],
                                            steps, prob, W4)
    assert J2 == J and np.array_equal(dk2, dk) and np.array_equal(lam2, lam0)


def test_field_solve_transpose_by_dot_product():
    rng = np.random.default_rng(12)
    nz, ny, nx = 7, 5, 6
    kbars = [igf.field_cell_average(nx, ny, nz, 1.0, 0.7, 2.3, a) for a in range(3)]
    Q = rng.standard_normal((nz, ny, nx))
    e = rng.standard_normal((3, nz, ny, nx))
    lhs = np.sum(pic.solve_field(Q, kbars) * e)
    rhs = np.sum(Q * adj.solve_field_T(e, kbars))
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)


@pytest.mark.parametrize("follow", [True, False])
@pytest.mark.parametrize("shape", [1, 2])
def test_direct_field_adjoint_matches_central_differences(shape, follow):
    n, steps = 300, 5
    c = workloads.SMALL
    prob = pic.make_problem(n, c.qm_qeeV, c.charge_C, c.kin_energy_MeV, c.mass_MeV, (10, 12, 12),
                            shape, direct_field=True)
    X0 = _beam(n, seed=13)
    geoms = None if follow else _frozen_elements(X0, THICK, steps, prob)
    J, dk, lam0, _ = adj.adjoint_elements(X0, THICK, steps, prob, W4, geoms=geoms)
    bar_k, bar_x = FD_BARS[follow]

    def J_of(els, X_=X0):
        XN, _ = adj.forward_elements(X_, els, steps, prob, geoms=geoms)
        return adj.objective(XN, W4)

    XN, _ = adj.forward_elements(X0, THICK, steps, prob)
    assert np.array_equal(XN, pic.track_elements(X0, THICK, steps, prob))
    for e in (1, 2, 3):
        h = 1e-6 * abs(THICK[e][1])

        def shifted(t, e=e):
            els = list(THICK)
            kind, k, ds, ns = els[e]
            els[e] = (kind, k + t, ds, ns)
            return J_of(els)

        assert abs(_fd(shifted, 0.0, h) - dk[e]) < bar_k * np.abs(dk).max(), e
    D = np.random.default_rng(14).standard_normal(X0.shape) * X0.std(axis=1)[:, None]
    fd = _fd(lambda t: J_of(THICK, X0 + t * D), 0.0, 1e-6)
    assert abs(fd - np.sum(lam0 * D)) < bar_x * abs(np.sum(lam0 * D)) + J_NOISE * abs(J) / 1e-6
