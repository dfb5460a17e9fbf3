"""pic_track_n_steps_binned (X left in the library's tile order, labels permuted with the
particles) against pic_track_n_steps from the same beam: particle by particle and bit for bit,
over several calls, for the binned path and for the gather's global-load fallback, and the
error contract (X untouched after a device error).  A run split into calls equals the same run
in one call to rounding."""
import numpy as np
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import paper_2208_02382_amd as p
    return p


def _beam(lib, cfg, tuning=None, grid_fp32=False, direct_field=False):
    b = lib.Beam(cfg.n, cfg.qm_qeeV, cfg.charge_C, cfg.kin_energy_MeV, cfg.mass_MeV, cfg.shape,
                 cfg.nodes, grid_fp32=grid_fp32, tuning=tuning, direct_field=direct_field)
    b.init(cfg.sigma_matrix, seed=cfg.seed, halo_frac=0.1)
    return b


def _compare(lib, cfg, lattice, calls, tuning=None, grid_fp32=False, direct_field=False):
    """Track the beam in caller-order calls and in binned calls of the given step counts, the
    latter with labels 0..n-1; the binned slot i must hold the caller-order particle ids[i].
    Both sides end their calls after the same steps: inside a call a slice's second half map
    and the next slice's first act as one product, at a call's end they are applied apart."""
    ref = _beam(lib, cfg, tuning, grid_fp32, direct_field)
    for k in calls:
        ref.track(lattice, k)
    Xc = ref.X.clone()
    assert ref.check() == lib.PIC_OK
    ref.close()
    b = _beam(lib, cfg, tuning, grid_fp32, direct_field)
    ids = torch.arange(cfg.n, dtype=torch.int32, device="cuda")
    for k in calls:
        b.track(lattice, k, binned=True, ids=ids)
    assert b.check() == lib.PIC_OK
    idl = ids.long()
    assert torch.equal(torch.sort(idl).values, torch.arange(cfg.n, device="cuda"))
    assert torch.equal(b.X, Xc[:, idl])
    # the binned order groups the particles by tile: far from the caller's order
    assert (idl[1:] < idl[:-1]).sum().item() > cfg.n // 100
    b.close()


@pytest.mark.parametrize("shape,grid_fp32", [(1, False), (2, False), (2, True)])
def test_binned_calls_equal_caller_order_tracking(lib, shape, grid_fp32):
    cfg = workloads.MEDIUM.with_(n=200_003, nodes=(32, 36, 48), shape=shape)
    # even step counts keep the two-element lattice in phase across calls
    _compare(lib, cfg, cfg.lattice, [2, 4, 2], grid_fp32=grid_fp32)


@pytest.mark.parametrize("binned", [False, True])
def test_a_run_split_into_calls_equals_one_call_to_rounding(lib, binned):
    # a call's last step applies the slice's second half map alone and the next call starts
    # with the next slice's first, where one call applies their product: the same linear maps,
    # rounded in another order
    cfg = workloads.MEDIUM.with_(n=200_003, nodes=(32, 36, 48), shape=2)
    one = _beam(lib, cfg)
    one.track(cfg.lattice, 8)
    split = _beam(lib, cfg)
    ids = torch.arange(cfg.n, dtype=torch.int32, device="cuda")
    for k in [2, 4, 2]:
        split.track(cfg.lattice, k, binned=binned, ids=ids if binned else None)
    assert one.check() == lib.PIC_OK and split.check() == lib.PIC_OK
    X1 = one.X.cpu().numpy()[:, ids.long().cpu().numpy()] if binned else one.X.cpu().numpy()
    Xs = split.X.cpu().numpy()
    rms = X1.std(axis=1)
    err = (np.abs(Xs - X1).max(axis=1) / rms).max()
    assert err < 1e-13, err
    one.close()
    split.close()


@pytest.mark.parametrize("calls", [[1], [1, 1], [3, 1, 2]])
def test_binned_calls_of_any_length(lib, calls):
    # a one-element lattice keeps every split of the steps in phase; a call's first step on a
    # beam that no binned call has ordered moves the particles into tile order (and a one-step
    # call then copies them out), later calls only rank
    cfg = workloads.MEDIUM.with_(n=120_000, nodes=(32, 32, 32), shape=2)
    _compare(lib, cfg, [(1.0, 0.5)], calls)


def test_binned_calls_at_a_size_that_takes_the_wide_staged_scatter(lib):
    # above 256 x 16384 particles the first step's move into tile order and the return to the
    # caller's order use the wide (16384-particle) staged scatter blocks
    cfg = workloads.MEDIUM.with_(n=4_300_001, nodes=(64, 64, 64), shape=2)
    _compare(lib, cfg, cfg.lattice, [2, 2])


def test_binned_thick_lattice_and_direct_field(lib):
    cfg = workloads.MEDIUM.with_(n=100_001, nodes=(32, 32, 32), shape=2)
    lattice = workloads.THICK_FODO
    # 125 slices per cell: one call ends inside an element, the next continues from there only
    # if the calls restart the cell, so every call here is a whole number of cells
    _compare(lib, cfg, lattice, [125, 125], direct_field=False)
    _compare(lib, cfg, [(2, 1.0, 1.0, 5), (2, -1.0, 1.0, 5)], [10, 10], direct_field=True)


def test_binned_gather_fallback_path(lib):
    # 18^3-node tiles: the TSC charge window (20^3 nodes, 64 KB) fits the LDS, the float64 field
    # window (192 KB) does not, so the gather-kick reads the field from global memory and the
    # state is copied back
    cfg = workloads.MEDIUM.with_(n=150_000, nodes=(36, 36, 36), shape=2)
    _compare(lib, cfg, cfg.lattice, [2, 2], tuning={"tile": (18, 18, 18)})


def test_binned_without_labels_keeps_the_moments(lib):
    cfg = workloads.MEDIUM.with_(n=200_000, nodes=(48, 48, 48))
    ref = _beam(lib, cfg)
    ref.track(cfg.lattice, 6)
    m_ref, c_ref = ref.moments()
    ref.close()
    b = _beam(lib, cfg)
    b.track(cfg.lattice, 4, binned=True)
    b.track(cfg.lattice, 2, binned=True)
    m, c = b.moments()
    c, c_ref = np.array(c), np.array(c_ref)
    # the same particles in another order: the reductions' rounding only
    assert np.abs(c - c_ref).max() <= 1e-13 * np.abs(c_ref).max()
    b.close()


def test_binned_call_leaves_x_on_a_device_error(lib):
    cfg = workloads.MEDIUM.with_(n=50_000, nodes=(32, 32, 32))
    b = _beam(lib, cfg)
    X = b.X
    X[0, 1234] = float("nan")
    before = X.clone()
    ids = torch.arange(cfg.n, dtype=torch.int32, device="cuda")
    b.track(cfg.lattice, 3, binned=True, ids=ids)
    assert b.check() == lib.PIC_EDOMAIN
    assert torch.equal(torch.isnan(b.X), torch.isnan(before))
    assert torch.equal(torch.nan_to_num(b.X), torch.nan_to_num(before))
    assert torch.equal(ids, torch.arange(cfg.n, dtype=torch.int32, device="cuda"))
    b.close()
