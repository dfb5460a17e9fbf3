"""GPU parity: every call of the C ABI against the CPU FP64 oracle on the same seeded inputs.

Tolerances (float64 paths): 1e-12 relative to the largest magnitude of the compared array
(grids, fields) or to the rms size of the coordinate (particles).  The two sides differ only
in rounding: the deposit's fixed-point rounding (every contribution is rounded to a multiple of
a power of two before the exact integer sums of pic_deposit and the tracking loop), the FFT's
operation order, libm against the device math library, and fused multiply-adds.
"""
import numpy as np
import pytest
import torch

import workloads
from oracle import pic as opic
from oracle import rng as orng

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def lib():
    import paper_2208_02382_amd as p
    return p


def _problem(cfg, n=None, nodes=None, shape=None):
    return opic.make_problem(cfg.n if n is None else n, cfg.qm_qeeV, cfg.charge_C,
                             cfg.kin_energy_MeV, cfg.mass_MeV,
                             cfg.nodes if nodes is None else nodes,
                             cfg.shape if shape is None else shape)


def _gpu_beam(lib, cfg, n, nodes, shape, grid_fp32=False, space_charge=True, tuning=None):
    return lib.Beam(n, cfg.qm_qeeV, cfg.charge_C, cfg.kin_energy_MeV, cfg.mass_MeV, shape, nodes,
                    grid_fp32=grid_fp32, space_charge=space_charge, tuning=tuning)


def _start(lib, cfg, n, nodes, shape, seed=None, **kw):
    """GPU beam and oracle X0 from the same seeded draws."""
    xi = workloads.draw_xi(cfg, n=n, seed=seed)
    b = _gpu_beam(lib, cfg, n, nodes, shape, **kw)
    b.init_from_normals(cfg.sigma_matrix, torch.from_numpy(xi).cuda())
    X0 = opic.init_from_normals(cfg.sigma_matrix, xi)
    return b, X0


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def _coord_err(Xg, Xo):
    sig = Xo.std(axis=1)
    return (np.abs(Xg - Xo).max(axis=1) / sig).max()


CASES = [  # (n, nodes, shape)
    (10_000, (32, 32, 32), 1),
    (10_007, (24, 18, 36), 2),
    (4_093, (16, 12, 24), 1),
]


def test_init_from_normals(lib):
    cfg = workloads.SMALL
    b, X0 = _start(lib, cfg, 10_007, cfg.nodes, 1)
    Xg = b.X.cpu().numpy()
    assert _coord_err(Xg, X0) < 1e-15


def test_init_philox_matches_oracle_generator(lib):
    cfg = workloads.LARGE
    n = 100_003
    nh = workloads.n_halo(n, cfg.halo_frac)
    b = _gpu_beam(lib, cfg, n, cfg.nodes, cfg.shape)
    b.init(cfg.sigma_matrix, seed=cfg.seed, halo_frac=cfg.halo_frac)
    Xg = b.X.cpu().numpy()
    X0 = opic.init_from_normals(cfg.sigma_matrix, orng.beam_xi(n, cfg.seed, nh))
    assert _coord_err(Xg, X0) < 1e-13
    # halo particles lie inside +-4 sigma
    s = np.sqrt(np.diag(cfg.sigma_matrix))
    assert np.all(np.abs(Xg[:, n - nh:]) <= 4 * s[:, None] * (1 + 1e-15))


@pytest.mark.parametrize("n,nodes,shape", CASES)
def test_deposit_solve_gather_push(lib, n, nodes, shape):
    cfg = workloads.SMALL
    b, X = _start(lib, cfg, n, nodes, shape)
    prob = _problem(cfg, n, nodes, shape)
    # first half of a step on both sides
    b.push(lib.PUSH_THINQUAD, 1.0)
    b.push(lib.PUSH_DRIFT, 0.25)
    X = opic.drift(opic.thin_quad(X, 1.0), 0.25, prob)
    assert _coord_err(b.X.cpu().numpy(), X) < 1e-15
    # deposit
    rho = b.deposit()
    geom = opic.geometry(X, prob)
    origin, h, h_rest = b.geometry()
    assert np.array_equal(origin, geom.origin) and np.array_equal(h, geom.h)
    assert np.array_equal(h_rest, geom.h_rest)
    Q = opic.deposit(X, geom, prob)
    assert _rel(rho.cpu().numpy(), Q) < TOL
    # Poisson solve and field
    phi = b.new_phi()
    _, E = b.poisson_solve(rho, phi=phi)
    phi_o = opic.solve(Q, opic.green(geom, prob))
    E_o = opic.field(phi_o, geom)
    assert _rel(phi.cpu().numpy(), phi_o) < TOL
    Eg = E.cpu().numpy()
    for c in range(3):
        assert _rel(Eg[c], E_o[c]) < TOL
    # gather
    Ep = b.gather(E)
    Ep_o = opic.gather(E_o, X, geom, prob)
    Epg = Ep.cpu().numpy()
    for c in range(3):
        assert _rel(Epg[c], Ep_o[c]) < TOL
    # kick and second half drift
    b.push(lib.PUSH_KICK, 0.5, Ep)
    b.push(lib.PUSH_DRIFT, 0.25)
    X = opic.drift(opic.kick(X, Ep_o, 0.5, prob), 0.25, prob)
    assert _coord_err(b.X.cpu().numpy(), X) < TOL
    assert b.check() == lib.PIC_OK


@pytest.mark.parametrize("n,nodes,shape", CASES[:2])
def test_track_n_steps_parity(lib, n, nodes, shape):
    cfg = workloads.SMALL
    b, X = _start(lib, cfg, n, nodes, shape)
    prob = _problem(cfg, n, nodes, shape)
    ks, dss = workloads.lattice_arrays(cfg)
    steps = 20
    b.track(cfg.lattice, steps)
    Xo = opic.track(X, ks, dss, steps, prob)
    Xg = b.X.cpu().numpy()
    assert _coord_err(Xg, Xo) < TOL
    mean, cov = b.moments()
    mo, covo, _ = opic.moments(Xo)
    assert np.abs(np.array(mean) - mo).max() < TOL * np.sqrt(np.diag(covo)).max()
    assert _rel(np.array(cov), covo) < TOL


def test_track_without_space_charge(lib):
    cfg = workloads.SMALL
    b, X = _start(lib, cfg, 5_000, cfg.nodes, 1, space_charge=False)
    prob = _problem(cfg, 5_000)
    ks, dss = workloads.lattice_arrays(cfg)
    b.track(cfg.lattice, 20)
    Xo = opic.track(X, ks, dss, 20, prob, space_charge=False)
    assert _coord_err(b.X.cpu().numpy(), Xo) < 1e-14


def test_fp32_grid_moments_within_1e5(lib):
    cfg = workloads.SMALL
    n = 10_000
    b, X = _start(lib, cfg, n, cfg.nodes, 1, grid_fp32=True)
    prob = _problem(cfg, n)
    ks, dss = workloads.lattice_arrays(cfg)
    b.track(cfg.lattice, 20)
    _, _, m_o = opic.moments(opic.track(X, ks, dss, 20, prob))
    mean, cov = b.moments()
    cov = np.array(cov)
    m_g = np.array([np.sqrt(cov[0, 0]), np.sqrt(cov[2, 2]),
                    np.sqrt(cov[0, 0] * cov[1, 1] - cov[0, 1] ** 2),
                    np.sqrt(cov[2, 2] * cov[3, 3] - cov[2, 3] ** 2)])
    assert np.all(np.abs(m_g - m_o) / m_o < 1e-5)


def test_device_errors_are_reported(lib):
    cfg = workloads.SMALL
    # a single particle has a zero-extent box
    b = _gpu_beam(lib, cfg, 1, (8, 8, 8), 1)
    b.init_from_normals(cfg.sigma_matrix, torch.zeros((6, 1), dtype=torch.float64, device="cuda"))
    b.deposit()
    assert b.check() == lib.PIC_EDOMAIN
    with pytest.raises(lib.PicError):
        b.moments()
    # a non-finite coordinate
    b2, _ = _start(lib, cfg, 1000, (8, 8, 8), 2)
    b2.X[0, 17] = float("nan")
    b2.track(cfg.lattice, 2)
    assert b2.check() == lib.PIC_EDOMAIN
    # re-initialising clears the flag
    b2.init_from_normals(cfg.sigma_matrix, torch.from_numpy(workloads.draw_xi(cfg, n=1000)).cuda())
    assert b2.check() == lib.PIC_OK


def test_zero_charge_equals_the_linear_map(lib):
    # a zero bunch charge deposits nothing: the space-charge kick vanishes and tracking reduces
    # to the linear maps of the lattice
    cfg = workloads.SMALL.with_(charge_C=0.0)
    n = 3_001
    b, X = _start(lib, cfg, n, (16, 16, 16), 2)
    prob = _problem(cfg, n, (16, 16, 16), 2)
    ks, dss = workloads.lattice_arrays(cfg)
    b.track(cfg.lattice, 6)
    Xo = opic.track(X, ks, dss, 6, prob, space_charge=False)
    assert _coord_err(b.X.cpu().numpy(), Xo) < 1e-14
    assert b.check() == lib.PIC_OK


@pytest.mark.parametrize("steps", [1, 2, 7])
def test_box_changing_severalfold_every_step(lib, steps):
    # thin quads of +-12/m over 0.5 m drifts change the beam's size several-fold every step,
    # so most particles change tile between steps
    cfg = workloads.SMALL.with_(lattice=((-12.0, 0.5), (12.0, 0.5)))
    n, nodes, shape = 6_007, (16, 24, 16), 2
    b, X = _start(lib, cfg, n, nodes, shape)
    b.track(cfg.lattice, steps)
    ks, dss = workloads.lattice_arrays(cfg)
    Xo = opic.track(X, ks, dss, steps, _problem(cfg, n, nodes, shape))
    assert _coord_err(b.X.cpu().numpy(), Xo) < TOL
    assert b.check() == lib.PIC_OK


LISTING = dict(sigmaX=3.9984884770e-5, sigmaY=3.9984884770e-5, sigmaT=1.0e-3,
               sigmaPx=2.6623538760e-5, sigmaPy=2.6623538760e-5, sigmaPt=2.0e-3,
               muxpx=-0.846574929020762, muypy=0.846574929020762, mutpt=0.0)


def test_init_waterbag_matches_oracle_generator(lib):
    cfg = workloads.MEDIUM
    n = 100_003
    S = np.array(lib.sigma_from_params(**LISTING))
    assert np.allclose(S, opic.sigma_from_params(**LISTING), rtol=1e-15, atol=0)
    b = _gpu_beam(lib, cfg, n, cfg.nodes, 1)
    b.init_waterbag(S, seed=31)
    Xg = b.X.cpu().numpy()
    X0 = opic.init_waterbag(S, orng.waterbag_xi(n, 31))
    assert _coord_err(Xg, X0) < 1e-13
    q = np.einsum("in,ij,jn->n", Xg, np.linalg.inv(S), Xg)
    assert q.max() <= 8.0 * (1 + 1e-9)


@pytest.mark.parametrize("space_charge", [False, True])
def test_listing_example_through_the_fodo_cell(lib, space_charge):
    # Listing 1: 1e4 macroparticles of a Waterbag beam, 2 GeV electrons, 1 nC, TSC, the FODO
    # cell of thick elements (125 slices)
    mass = 0.510998950
    n, nodes, shape, steps = 10_000, (16, 16, 16), 2, 125
    S = opic.sigma_from_params(**LISTING)
    b = lib.Beam(n, -1.0e-6 / mass, 1.0e-9, 2.0e3, mass, shape, nodes,
                 space_charge=space_charge)
    b.init_waterbag(S, seed=5)
    X0 = b.X.cpu().numpy()
    b.track(workloads.THICK_FODO, steps)
    prob = opic.make_problem(n, -1.0e-6 / mass, 1.0e-9, 2.0e3, mass, nodes, shape)
    Xo = opic.track_elements(X0, workloads.THICK_FODO, steps, prob, space_charge=space_charge)
    Xg = b.X.cpu().numpy()
    assert _coord_err(Xg, Xo) < (TOL if space_charge else 3e-13)
    if not space_charge:
        # the paper's benchmark criterion: the emittances stay constant through the cell
        _, _, m0 = opic.moments(X0)
        _, _, m1 = opic.moments(Xg)
        assert np.all(np.abs(m1[2:] - m0[2:]) / m0[2:] < 1e-12)
