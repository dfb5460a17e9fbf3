"""GPU parity of batched tracking: beams of different particle counts and grids, tracked by one
graph launch, against the CPU FP64 oracle run beam by beam and against the single-beam path.

Tolerances as for single beams: 1e-12 of each coordinate's rms (float64 grids); rms size and
emittance within 1e-5 relative for float32 grids.
"""
import ctypes

import numpy as np
import pytest
import torch

import workloads
from oracle import pic as opic

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def lib():
    import paper_2208_02382_amd as p
    return p


# (n, nodes, k): particle counts and grids differ between beams, including a ragged grid
MIX = [(3_001, (16, 16, 16), 0.7), (12_000, (32, 32, 32), 1.9), (4_093, (12, 18, 24), 1.2),
       (7_777, (24, 24, 24), 0.5), (2_048, (48, 48, 48), 1.5)]


def _cfg(n, nodes, k, b):
    return workloads.MEDIUM.with_(n=n, nodes=nodes, lattice=((k, 0.5), (-k, 0.5)), seed=1000 + b)


def _problem(cfg, shape):
    return opic.make_problem(cfg.n, cfg.qm_qeeV, cfg.charge_C, cfg.kin_energy_MeV, cfg.mass_MeV,
                             cfg.nodes, shape)


def _beams(lib, shape, grid_fp32=False, mix=MIX):
    cfgs = [_cfg(n, nodes, k, b) for b, (n, nodes, k) in enumerate(mix)]
    gpu, X0 = [], []
    for c in cfgs:
        xi = workloads.draw_xi(c)
        g = lib.Beam(c.n, c.qm_qeeV, c.charge_C, c.kin_energy_MeV, c.mass_MeV, shape, c.nodes,
                     grid_fp32=grid_fp32)
        g.init_from_normals(c.sigma_matrix, torch.from_numpy(xi).cuda())
        gpu.append(g)
        X0.append(opic.init_from_normals(c.sigma_matrix, xi))
    return cfgs, gpu, X0


def _coord_err(Xg, Xo):
    return (np.abs(Xg - Xo).max(axis=1) / Xo.std(axis=1)).max()


def _rms(cov):
    cov = np.asarray(cov)
    return np.array([np.sqrt(cov[0, 0]), np.sqrt(cov[2, 2]),
                     np.sqrt(cov[0, 0] * cov[1, 1] - cov[0, 1] ** 2),
                     np.sqrt(cov[2, 2] * cov[3, 3] - cov[2, 3] ** 2)])


@pytest.mark.parametrize("shape", [1, 2])
def test_batch_matches_oracle_and_replays(lib, shape):
    cfgs, gpu, X0 = _beams(lib, shape)
    batch = lib.Batch(gpu, [c.lattice for c in cfgs])
    steps = 7
    batch.track(steps)
    torch.cuda.synchronize()
    assert batch.check() == [lib.PIC_OK] * len(gpu)
    Xo = []
    for c, g, X in zip(cfgs, gpu, X0):
        ks, dss = workloads.lattice_arrays(c)
        Xo.append(opic.track(X, ks, dss, steps, _problem(c, shape)))
        assert _coord_err(g.X.cpu().numpy(), Xo[-1]) < TOL, c.nodes
    # the second call replays the captured graph from the state the first one left
    batch.track(steps)
    torch.cuda.synchronize()
    for c, g, X in zip(cfgs, gpu, Xo):
        ks, dss = workloads.lattice_arrays(c)
        ref = opic.track(X, ks, dss, steps, _problem(c, shape))
        assert _coord_err(g.X.cpu().numpy(), ref) < TOL, c.nodes
    batch.close()


def test_batch_matches_single_beam_path(lib):
    cfgs, gpu, _ = _beams(lib, 1)
    _, single, _ = _beams(lib, 1)
    batch = lib.Batch(gpu, [c.lattice for c in cfgs])
    batch.track(12)
    for c, s in zip(cfgs, single):
        s.track(c.lattice, 12)
    torch.cuda.synchronize()
    for g, s in zip(gpu, single):
        # the same kernels' arithmetic and order-independent charge grids: the same bits
        assert torch.equal(g.X, s.X)


def test_batch_fp32_grid_moments_within_1e5(lib):
    mix = [(10_000, (32, 32, 32), 1.0), (6_000, (48, 48, 48), 1.7), (8_000, (16, 24, 32), 0.6)]
    cfgs, gpu, X0 = _beams(lib, 1, grid_fp32=True, mix=mix)
    batch = lib.Batch(gpu, [c.lattice for c in cfgs])
    batch.track(10)
    torch.cuda.synchronize()
    for c, g, X in zip(cfgs, gpu, X0):
        ks, dss = workloads.lattice_arrays(c)
        _, _, m_o = opic.moments(opic.track(X, ks, dss, 10, _problem(c, 1)))
        _, cov = g.moments()
        assert np.all(np.abs(_rms(cov) - m_o) / m_o < 1e-5)


def test_batch_device_error_stays_in_its_beam(lib):
    cfgs, gpu, X0 = _beams(lib, 1, mix=MIX[:3])
    gpu[1].X[2, 5] = float("nan")
    batch = lib.Batch(gpu, [c.lattice for c in cfgs])
    batch.track(3)
    torch.cuda.synchronize()
    assert batch.check() == [lib.PIC_OK, lib.PIC_EDOMAIN, lib.PIC_OK]
    for b in (0, 2):
        ks, dss = workloads.lattice_arrays(cfgs[b])
        ref = opic.track(X0[b], ks, dss, 3, _problem(cfgs[b], 1))
        assert _coord_err(gpu[b].X.cpu().numpy(), ref) < TOL


def test_batch_argument_errors(lib):
    cfgs, gpu, _ = _beams(lib, 1, mix=MIX[:2])
    tsc = lib.Beam(1000, cfgs[0].qm_qeeV, cfgs[0].charge_C, cfgs[0].kin_energy_MeV,
                   cfgs[0].mass_MeV, 2, (16, 16, 16))
    with pytest.raises(lib.PicError):
        lib.Batch([gpu[0], tsc], [cfgs[0].lattice, cfgs[0].lattice])
    batch = lib.Batch(gpu, [c.lattice for c in cfgs])
    # graph capture needs a stream other than the null stream
    assert lib._lib.pic_track_batch(batch._h, 3, None) == lib.PIC_EINVAL
    assert lib._lib.pic_track_batch(batch._h, 0, ctypes.c_void_p(batch.stream.cuda_stream)) \
        == lib.PIC_EINVAL
