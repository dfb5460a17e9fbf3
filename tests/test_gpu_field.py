"""GPU parity of the direct-field solve (E' from the integrated Green's functions of the field
itself, pic_beam_desc.direct_field = 1) against the oracle's solve_field, on the same seeded
inputs: the kernels' spectra and the three convolutions at 1e-12 of the largest field value,
whole tracking runs at 1e-12 of the rms size per coordinate, FP32 grids within 1e-5 in the rms
moments, the reverse sweep through the transposed field solve at 1e-12, and the rejection by
batches.  At the headline grid (128^3,
TSC) with the bench's launch shapes: one step on 2e6 particles, sampled particles against the
oracle within 1e-12.
"""
import numpy as np
import pytest
import torch

import workloads
from margins import check, rel_max
from oracle import pic as opic

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def lib():
    import paper_2208_02382_amd as p
    return p


def _problem(cfg, n, nodes, shape):
    return opic.make_problem(n, cfg.qm_qeeV, cfg.charge_C, cfg.kin_energy_MeV, cfg.mass_MeV,
                             nodes, shape, direct_field=True)


def _start(lib, cfg, n, nodes, shape, grid_fp32=False):
    xi = workloads.draw_xi(cfg, n=n)
    b = lib.Beam(n, cfg.qm_qeeV, cfg.charge_C, cfg.kin_energy_MeV, cfg.mass_MeV, shape, nodes,
                 grid_fp32=grid_fp32, direct_field=True)
    b.init_from_normals(cfg.sigma_matrix, torch.from_numpy(xi).cuda())
    return b, opic.init_from_normals(cfg.sigma_matrix, xi)


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def _coord_err(Xg, Xo):
    return (np.abs(Xg - Xo).max(axis=1) / Xo.std(axis=1)).max()


CASES = [  # (n, nodes, shape): several FFT tiles, ragged and non-power-of-two grids
    (10_000, (32, 32, 32), 1),
    (10_007, (24, 18, 36), 2),
    (4_093, (16, 12, 24), 1),
]


@pytest.mark.parametrize("n,nodes,shape", CASES)
def test_direct_field_solve_and_gather(lib, n, nodes, shape):
    cfg = workloads.SMALL
    b, X = _start(lib, cfg, n, nodes, shape)
    prob = _problem(cfg, n, nodes, shape)
    rho = b.deposit()
    geom = opic.geometry(X, prob)
    Q = opic.deposit(X, geom, prob)
    assert _rel(rho.cpu().numpy(), Q) < TOL
    # the field alone, then field and potential in one call
    _, E = b.poisson_solve(rho)
    E_o = opic.solve_field(Q, opic.green_field(geom, prob))
    Eg = E.cpu().numpy()
    for c in range(3):
        assert _rel(Eg[c], E_o[c]) < TOL, c
    phi = b.new_phi()
    _, E2 = b.poisson_solve(rho, phi=phi)
    assert _rel(phi.cpu().numpy(), opic.solve(Q, opic.green(geom, prob))) < TOL
    assert np.array_equal(E2.cpu().numpy(), Eg)
    Ep = b.gather(E).cpu().numpy()
    Ep_o = opic.gather(E_o, X, geom, prob)
    for c in range(3):
        assert _rel(Ep[c], Ep_o[c]) < TOL, c


@pytest.mark.parametrize("n,nodes,shape", CASES[:2])
def test_direct_field_tracking(lib, n, nodes, shape):
    cfg = workloads.SMALL
    b, X = _start(lib, cfg, n, nodes, shape)
    prob = _problem(cfg, n, nodes, shape)
    ks, dss = workloads.lattice_arrays(cfg)
    steps = 20
    b.track(cfg.lattice, steps)
    Xo = opic.track(X, ks, dss, steps, prob)
    assert _coord_err(b.X.cpu().numpy(), Xo) < TOL
    assert b.check() == lib.PIC_OK


def test_direct_field_differs_from_differenced_potential(lib):
    # the two readings of E' differ by the centred differences' O(h^2) error: well above the
    # parity tolerance, so the tracking test above could not pass on the potential's path
    cfg = workloads.SMALL
    n, nodes, shape = CASES[0]
    b, X = _start(lib, cfg, n, nodes, shape)
    ks, dss = workloads.lattice_arrays(cfg)
    b.track(cfg.lattice, 20)
    prob_phi = opic.make_problem(n, cfg.qm_qeeV, cfg.charge_C, cfg.kin_energy_MeV, cfg.mass_MeV,
                                 nodes, shape)
    Xphi = opic.track(X, ks, dss, 20, prob_phi)
    assert _coord_err(b.X.cpu().numpy(), Xphi) > 1e3 * TOL


def test_direct_field_fp32_grid_moments_within_1e5(lib):
    cfg = workloads.SMALL
    n, nodes, shape = CASES[0]
    b, X = _start(lib, cfg, n, nodes, shape, grid_fp32=True)
    prob = _problem(cfg, n, nodes, shape)
    ks, dss = workloads.lattice_arrays(cfg)
    b.track(cfg.lattice, 20)
    _, _, m_o = opic.moments(opic.track(X, ks, dss, 20, prob))
    _, cov = b.moments()
    cov = np.array(cov)
    m_g = np.array([np.sqrt(cov[0, 0]), np.sqrt(cov[2, 2]),
                    np.sqrt(cov[0, 0] * cov[1, 1] - cov[0, 1] ** 2),
                    np.sqrt(cov[2, 2] * cov[3, 3] - cov[2, 3] ** 2)])
    assert np.all(np.abs(m_g - m_o) / m_o < 1e-5)


def test_direct_field_through_thick_elements(lib):
    cfg = workloads.SMALL
    n, nodes, shape = CASES[1]
    b, X = _start(lib, cfg, n, nodes, shape)
    prob = _problem(cfg, n, nodes, shape)
    lat = [(lib.ELEM_DRIFT, 0.0, 0.25, 2), (lib.ELEM_QUAD, 1.0, 0.5, 3),
           (lib.ELEM_DRIFT, 0.0, 0.25, 2)]
    b.track(lat, 14)
    els = [(opic.DRIFT, 0.0, 0.25, 2), (opic.QUAD, 1.0, 0.5, 3), (opic.DRIFT, 0.0, 0.25, 2)]
    Xo = opic.track_elements(X, els, 14, prob)
    assert _coord_err(b.X.cpu().numpy(), Xo) < TOL


def test_batch_rejects_the_direct_field(lib):
    cfg = workloads.SMALL
    n, nodes, shape = CASES[0]
    b, _ = _start(lib, cfg, n, nodes, shape)
    with pytest.raises(lib.PicError) as e:
        lib.Batch([b], [cfg.lattice])
    assert e.value.status == lib.PIC_EUNSUPPORTED


@pytest.mark.parametrize("shape,ck", [(1, 3), (2, 2)])
def test_reverse_sweep_with_the_direct_field(lib, shape, ck):
    # the charge's adjoint through the transposed field convolutions; a lattice of thick and
    # thin elements
    from oracle import adjoint as oadj
    cfg = workloads.SMALL
    n, nodes, steps = 2_000, (12, 16, 18), 7
    lat = [(1, 0.0, 0.3, 2), (2, 1.4, 0.6, 3), (0, -0.6, 0.4, 1)]
    w = np.array([0.7, -0.4, 1.3, 0.9])
    b, X0 = _start(lib, cfg, n, nodes, shape)
    m, dk, lam, _ = b.track_adjoint(lat, steps, w, ckpt_every=ck)
    J, dk_o, lam_o, _ = oadj.adjoint_elements(X0, lat, steps, _problem(cfg, n, nodes, shape), w)
    assert abs(float(np.dot(w, m)) - J) < 1e-12 * abs(J)
    check("field-adjoint-dk", rel_max(dk, dk_o, np.abs(dk_o).max()), 1e-12)
    lg = lam.cpu().numpy()
    for r in range(6):
        scale = np.abs(lam_o[r]).max()
        if scale > 0:
            check("field-adjoint-lam%d" % r, rel_max(lg[r], lam_o[r], scale), 1e-12)


@pytest.mark.timeout(900)
def test_headline_grid_one_step_on_sampled_particles(lib):
    # the headline grid (128^3, TSC, Gaussian core with halo) and the bench's tuned launch
    # shapes, at 2e6 particles: the field kernels' spectra and convolutions depend on the grid
    # alone; the particle kernels are the potential path's, checked at 1e8 elsewhere
    from paper_2208_02382_amd import autotune
    cfg = workloads.LARGE
    n = 2_000_000
    tuning = autotune.lookup(cfg.n, cfg.nodes, cfg.shape, False)
    b = lib.Beam(n, cfg.qm_qeeV, cfg.charge_C, cfg.kin_energy_MeV, cfg.mass_MeV, cfg.shape,
                 cfg.nodes, tuning=tuning, direct_field=True)
    b.init(cfg.sigma_matrix, seed=cfg.seed, halo_frac=cfg.halo_frac)
    X0 = b.X.cpu().numpy()
    b.track(cfg.lattice, 1)
    X1 = b.X.cpu().numpy()
    assert b.check() == lib.PIC_OK
    b.close()
    prob = _problem(cfg, n, cfg.nodes, cfg.shape)
    k, L = cfg.lattice[0]
    X2 = opic.drift(opic.thin_quad(X0, k), 0.5 * L, prob)
    geom = opic.geometry(X2, prob)
    E = opic.solve_field(opic.deposit(X2, geom, prob), opic.green_field(geom, prob))
    S = np.random.default_rng(12).choice(n, 2000, replace=False)
    Xs = X2[:, S]
    Xo = opic.drift(opic.kick(Xs, opic.gather(E, Xs, geom, prob), L, prob), 0.5 * L, prob)
    scale = X1.std(axis=1)
    assert (np.abs(X1[:, S] - Xo).max(axis=1) / scale).max() < TOL
