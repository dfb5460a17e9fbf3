"""Bitwise reproducibility of the tracking loop: the binned deposit sums every tile's window as
64-bit integers (exact in any order) and forms the charge grid from them in a fixed order, the
reductions (box, moments) have a fixed shape, and every particle's gather and push is its own.
Two runs from the same state therefore give the same bits, although the order in which the
ranking places particles within a tile, and the order of the atomics, differ between runs.
The same holds across launch shapes that change the tiles' chunking but not the tiles.  (The
fused slice-step diagnostics sum in floating point over the particles each workgroup holds, so
they reproduce to rounding, not bit for bit.)"""
import numpy as np
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import paper_2208_02382_amd as p
    return p


def _beam(lib, cfg, n, nodes, shape, xi, **kw):
    b = lib.Beam(n, cfg.qm_qeeV, cfg.charge_C, cfg.kin_energy_MeV, cfg.mass_MeV, shape, nodes, **kw)
    b.init_from_normals(cfg.sigma_matrix, xi)
    return b


@pytest.mark.parametrize("grid_fp32", [False, True])
@pytest.mark.parametrize("shape", [1, 2])
def test_two_runs_give_the_same_bits(lib, grid_fp32, shape):
    cfg = workloads.SMALL
    n, nodes = 30_011, (24, 18, 36)
    xi = torch.from_numpy(workloads.draw_xi(cfg, n=n)).cuda()
    out = []
    for _ in range(2):
        b = _beam(lib, cfg, n, nodes, shape, xi, grid_fp32=grid_fp32,
                  tuning={"tile": (4, 4, 4), "chunk": 2048})
        b.track(cfg.lattice, 12)
        assert b.check() == lib.PIC_OK
        out.append(b.X.clone())
    assert torch.equal(out[0], out[1])


def test_chunk_size_and_workgroups_do_not_change_the_bits(lib):
    cfg = workloads.SMALL
    n, nodes, shape = 20_000, (32, 32, 32), 2
    xi = torch.from_numpy(workloads.draw_xi(cfg, n=n)).cuda()
    out = []
    for tun in ({"tile": (8, 8, 4), "chunk": 2048, "blocks": 64, "threads": 256},
                {"tile": (8, 8, 4), "chunk": 16384, "blocks": 1024, "threads": 1024,
                 "deposit_threads": 128}):
        b = _beam(lib, cfg, n, nodes, shape, xi, tuning=tun)
        b.track(cfg.lattice, 10)
        out.append(b.X.clone())
    assert torch.equal(out[0], out[1])


def test_batch_runs_give_the_same_bits(lib):
    # two batches of the same beams, one after the other; the first batch and its beams are torn
    # down (Python's rebinding: after the second batch is created) before the second batch's
    # first track() captures its graph, and the second batch is released right after its launch
    # with no synchronisation (its teardown waits for the launch)
    mix = [(7_001, (16, 16, 16), 1.0), (12_000, (24, 24, 24), 1.6), (3_000, (12, 18, 24), 0.7)]
    out = []
    batch = None
    for it in range(2):
        beams, lats = [], []
        for j, (n, nodes, k) in enumerate(mix):
            cfg = workloads.MEDIUM.with_(n=n, nodes=nodes, lattice=((k, 0.5), (-k, 0.5)))
            xi = torch.from_numpy(workloads.draw_xi(cfg, n=n, seed=50 + j)).cuda()
            beams.append(_beam(lib, cfg, n, nodes, 2, xi))
            lats.append(cfg.lattice)
        batch = lib.Batch(beams, lats)
        batch.track(8)
        if it == 1:
            batch.close()
        torch.cuda.synchronize()
        assert all(b.check() == lib.PIC_OK for b in beams)
        out.append([b.X.clone() for b in beams])
    for a, b in zip(*out):
        assert torch.equal(a, b)


@pytest.mark.parametrize("grid_fp32", [False, True])
def test_pic_deposit_gives_the_same_bits(lib, grid_fp32):
    cfg = workloads.SMALL
    n, nodes, shape = 50_003, (24, 18, 36), 2
    xi = torch.from_numpy(workloads.draw_xi(cfg, n=n)).cuda()
    b = _beam(lib, cfg, n, nodes, shape, xi, grid_fp32=grid_fp32)
    r1 = b.deposit().clone()
    # a different particle order gives the same charge grid, bit for bit
    perm = torch.randperm(n, generator=torch.Generator().manual_seed(5)).cuda()
    b2 = _beam(lib, cfg, n, nodes, shape, xi[:, perm].contiguous(), grid_fp32=grid_fp32)
    r2 = b2.deposit().clone()
    assert torch.equal(r1, b.deposit())
    assert torch.equal(r1, r2)
