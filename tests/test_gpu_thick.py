"""GPU parity of thick elements (drifts and quadrupoles of finite length, cut into slices, each
slice a half map, the space-charge kick over the slice length, and a second half map) against
the oracle's sliced tracking.

Tolerances: 1e-12 of each coordinate's rms with space charge (rounding only, as for thin
lattices).  Without space charge every slice is two products of 2x2 matrices whose cos/sin
and cosh/sinh entries each side computes with its own math library: rounding then grows
linearly with the number of half maps, a few ulp each, times the ratio of the largest
coordinate to its rms (about 4); 280 half maps give 3e-13.
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
                             nodes, shape)


def _start(lib, cfg, n, nodes, shape, seed=None, space_charge=True, tuning=None):
    xi = workloads.draw_xi(cfg, n=n, seed=seed)
    b = lib.Beam(n, cfg.qm_qeeV, cfg.charge_C, cfg.kin_energy_MeV, cfg.mass_MeV, shape, nodes,
                 space_charge=space_charge, tuning=tuning)
    b.init_from_normals(cfg.sigma_matrix, torch.from_numpy(xi).cuda())
    return b, opic.init_from_normals(cfg.sigma_matrix, xi)


def _coord_err(Xg, Xo):
    return (np.abs(Xg - Xo).max(axis=1) / Xo.std(axis=1)).max()


# 60 slices of the 125 in a cell: the first drift, the focusing quadrupole and part of the
# middle drift, so that both element boundaries kinds (drift to quad, quad to drift) are crossed
@pytest.mark.parametrize("n,nodes,shape,steps", [(5_000, (16, 16, 16), 2, 60),
                                                 (4_093, (12, 18, 24), 1, 60)])
def test_thick_fodo_with_space_charge(lib, n, nodes, shape, steps):
    cfg = workloads.SMALL
    b, X = _start(lib, cfg, n, nodes, shape)
    b.track(workloads.THICK_FODO, steps)
    Xo = opic.track_elements(X, workloads.THICK_FODO, steps, _problem(cfg, n, nodes, shape))
    assert _coord_err(b.X.cpu().numpy(), Xo) < TOL
    assert b.check() == lib.PIC_OK


def test_thick_fodo_cell_without_space_charge(lib):
    # a whole cell (125 slices) and the start of the next one
    cfg = workloads.SMALL
    n = 3_001
    b, X = _start(lib, cfg, n, (8, 8, 8), 1, space_charge=False)
    b.track(workloads.THICK_FODO, 140)
    Xo = opic.track_elements(X, workloads.THICK_FODO, 140, _problem(cfg, n, (8, 8, 8), 1),
                             space_charge=False)
    assert _coord_err(b.X.cpu().numpy(), Xo) < 3e-13


def test_mixed_thin_and_thick_elements(lib):
    # thin kicks between thick quadrupoles, one slice and several, and a zero-length drift
    lat = ((0, 0.4, 0.2, 1), (2, -0.8, 0.6, 3), (1, 0.0, 0.0, 2), (2, 1.3, 0.3, 1), (0.5, 0.25))
    cfg = workloads.SMALL
    n, nodes, shape = 6_000, (16, 24, 16), 2
    b, X = _start(lib, cfg, n, nodes, shape, seed=77)
    steps = 17
    b.track(lat, steps)
    elems = [e if len(e) == 4 else (0, e[0], e[1], 1) for e in lat]
    Xo = opic.track_elements(X, elems, steps, _problem(cfg, n, nodes, shape))
    assert _coord_err(b.X.cpu().numpy(), Xo) < TOL


def test_thin_element_form_equals_pair_form(lib):
    cfg = workloads.SMALL
    n, nodes = 2_000, (16, 16, 16)
    b1, _ = _start(lib, cfg, n, nodes, 1)
    b2, _ = _start(lib, cfg, n, nodes, 1)
    b1.track(cfg.lattice, 6)
    b2.track([(0, k, ds, 1) for k, ds in cfg.lattice], 6)
    # the same arithmetic, and the tracking loop's charge grid does not depend on the order of
    # the particles or of the atomics: equal bit for bit
    assert torch.equal(b1.X, b2.X)


def test_batch_with_thin_and_thick_lattices(lib):
    lats = [workloads.THICK_FODO, ((1.0, 0.5), (-1.0, 0.5)),
            ((2, 0.9, 0.8, 4), (1, 0.0, 0.4, 2), (2, -0.9, 0.8, 4), (1, 0.0, 0.4, 2))]
    mix = [(3_001, (16, 16, 16)), (5_000, (24, 24, 24)), (2_500, (12, 18, 24))]
    cfg = workloads.MEDIUM
    shape = 2
    beams, X0, cfgs = [], [], []
    for i, (n, nodes) in enumerate(mix):
        c = cfg.with_(n=n, nodes=nodes, seed=500 + i)
        b, X = _start(lib, c, n, nodes, shape)
        beams.append(b)
        X0.append(X)
        cfgs.append(c)
    steps = 12
    batch = lib.Batch(beams, lats)
    batch.track(steps)
    torch.cuda.synchronize()
    assert all(st == lib.PIC_OK for st in batch.check())
    for b, X, c, lat in zip(beams, X0, cfgs, lats):
        elems = [e if len(e) == 4 else (0, e[0], e[1], 1) for e in lat]
        Xo = opic.track_elements(X, elems, steps, _problem(c, c.n, c.nodes, shape))
        assert _coord_err(b.X.cpu().numpy(), Xo) < TOL
    batch.close()
    for b in beams:
        b.close()


# drifts, quadrupoles of either sign (one weak enough, |k| (l/2)^2 < 0.1, for the series form
# of the strength derivative) and a thin element, cut into slices
ADJ_LATTICE = [(1, 0.0, 0.3, 2), (2, 1.4, 0.6, 3), (0, -0.6, 0.4, 1), (2, -1.1, 0.5, 2),
               (2, 0.05, 0.6, 2)]


@pytest.mark.parametrize("shape,steps,ck", [(1, 11, 4), (2, 9, 3)])
def test_reverse_sweep_through_thick_elements(lib, shape, steps, ck):
    from oracle import adjoint as oadj
    cfg = workloads.SMALL
    n, nodes = 2_500, (12, 16, 18)
    w = np.array([0.7, -0.4, 1.3, 0.9])
    b, X0 = _start(lib, cfg, n, nodes, shape)
    m, dk, lam, _ = b.track_adjoint(ADJ_LATTICE, steps, w, ckpt_every=ck)
    J, dk_o, lam_o, _ = oadj.adjoint_elements(X0, ADJ_LATTICE, steps,
                                              _problem(cfg, n, nodes, shape), w)
    assert abs(float(np.dot(w, m)) - J) < 1e-12 * abs(J)
    assert dk[0] == 0.0
    check("thick-adjoint-dk", rel_max(dk, dk_o, np.abs(dk_o).max()), 1e-12)
    lg = lam.cpu().numpy()
    for r in range(6):
        scale = np.abs(lam_o[r]).max()
        if scale > 0:
            check("thick-adjoint-lam%d" % r, rel_max(lg[r], lam_o[r], scale), 1e-12)
    # X holds the final state of the forward run, as pic_track_n_steps leaves it
    Xo = opic.track_elements(X0, ADJ_LATTICE, steps, _problem(cfg, n, nodes, shape))
    assert _coord_err(b.X.cpu().numpy(), Xo) < TOL


def _diag_oracle(X, elements, steps, prob, space_charge=True):
    sl = opic.slices(elements)
    out = []
    for j in range(steps):
        kind, k, ell = sl[j % len(sl)]
        X = opic.slice_step(X, kind, k, ell, prob, space_charge)
        mean, cov, _ = opic.moments(X)
        out.append(np.concatenate([mean, cov[np.triu_indices(6)]]))
    return X, np.array(out)


@pytest.mark.parametrize("space_charge,tuning", [(True, None), (False, None),
                                                 (True, {"tile": (16, 16, 12)})])
def test_slice_step_diagnostics(lib, space_charge, tuning):
    # the third case's field window (18 x 18 x 14 nodes, 109 KB in float64) fits; a tile of
    # (16, 16, 16) would not, see the next test
    cfg = workloads.SMALL
    n, nodes, shape, steps = 5_000, (16, 16, 16), 2, 30
    b, X = _start(lib, cfg, n, nodes, shape, space_charge=space_charge, tuning=tuning)
    b2, _ = _start(lib, cfg, n, nodes, shape, space_charge=space_charge, tuning=tuning)
    diag = b.track(workloads.THICK_FODO, steps, diagnostics=True).cpu().numpy()
    b2.track(workloads.THICK_FODO, steps)
    assert diag.shape == (steps, 27)
    Xo, do = _diag_oracle(X, workloads.THICK_FODO, steps, _problem(cfg, n, nodes, shape),
                          space_charge)
    rms = np.sqrt(np.diag(np.cov(Xo)))
    assert np.all(np.abs(diag[:, :6] - do[:, :6]) / rms < TOL)
    assert np.abs(diag[:, 6:] - do[:, 6:]).max() < TOL * np.abs(do[:, 6:]).max()
    # the end state equals tracking without diagnostics (the same arithmetic, split in two
    # passes at the end of each step)
    assert _coord_err(b.X.cpu().numpy(), b2.X.cpu().numpy()) < 1e-13
    assert _coord_err(b.X.cpu().numpy(), Xo) < TOL


@pytest.mark.parametrize("offset_sigmas", [0.0, 30.0])
def test_slice_step_diagnostics_of_an_offset_beam(lib, offset_sigmas):
    # the moments are summed about a shift inside the gather-kick (the grid centre on the first
    # step, the previous step's means after it): a beam centred 30 sigma off axis in x, px, y
    # and delta keeps the centred moments at the parity bar
    cfg = workloads.SMALL
    n, nodes, shape, steps = 4_001, (16, 12, 16), 1, 12
    b, X = _start(lib, cfg, n, nodes, shape)
    off = offset_sigmas * np.sqrt(np.diag(np.array(cfg.sigma_matrix)))
    off[3] = off[4] = 0.0
    for r in range(6):
        b.X[r] += float(off[r])
    X = X + off[:, None]
    diag = b.track(workloads.THICK_FODO, steps, diagnostics=True).cpu().numpy()
    _, do = _diag_oracle(X, workloads.THICK_FODO, steps, _problem(cfg, n, nodes, shape))
    rms = np.sqrt(np.diag(np.cov(X)))
    assert np.all(np.abs(diag[:, :6] - do[:, :6]) / rms < TOL)
    assert np.abs(diag[:, 6:] - do[:, 6:]).max() < TOL * np.abs(do[:, 6:]).max()


def test_slice_step_diagnostics_with_the_unbinned_gather(lib):
    # a (24, 18, 18) tile needs a 250 KB field window, beyond LDS: the gather-kick runs
    # unbinned, stops at the end of the step, and separate passes take the moments and apply
    # the next first half map
    cfg = workloads.SMALL
    n, nodes, shape, steps = 4_001, (24, 18, 36), 2, 14
    tun = {"tile": (24, 18, 18)}
    b, X = _start(lib, cfg, n, nodes, shape, tuning=tun)
    diag = b.track(workloads.THICK_FODO, steps, diagnostics=True).cpu().numpy()
    Xo, do = _diag_oracle(X, workloads.THICK_FODO, steps, _problem(cfg, n, nodes, shape))
    rms = np.sqrt(np.diag(np.cov(Xo)))
    assert np.all(np.abs(diag[:, :6] - do[:, :6]) / rms < TOL)
    assert np.abs(diag[:, 6:] - do[:, 6:]).max() < TOL * np.abs(do[:, 6:]).max()
    assert _coord_err(b.X.cpu().numpy(), Xo) < TOL
