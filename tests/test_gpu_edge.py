"""GPU edge cases against the oracle: beams smaller than a wavefront and a ragged last
wavefront, the largest grid the FFT plan accepts along one axis (512-point padded transforms),
radix-3 grid sizes, the largest tile count, and a beam with zero extent along one axis (an error
state, not a result)."""
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


def _run(lib, n, nodes, shape, steps, tuning=None, cfg=workloads.SMALL, seed=None):
    xi = workloads.draw_xi(cfg, n=n, seed=seed)
    b = lib.Beam(n, cfg.qm_qeeV, cfg.charge_C, cfg.kin_energy_MeV, cfg.mass_MeV, shape, nodes,
                 tuning=tuning)
    b.init_from_normals(cfg.sigma_matrix, torch.from_numpy(xi).cuda())
    X0 = opic.init_from_normals(cfg.sigma_matrix, xi)
    b.track(cfg.lattice, steps)
    assert b.check() == lib.PIC_OK
    prob = opic.make_problem(n, cfg.qm_qeeV, cfg.charge_C, cfg.kin_energy_MeV, cfg.mass_MeV,
                             nodes, shape)
    ks, dss = workloads.lattice_arrays(cfg)
    Xo = opic.track(X0, ks, dss, steps, prob)
    Xg = b.X.cpu().numpy()
    return (np.abs(Xg - Xo).max(axis=1) / Xo.std(axis=1)).max()


@pytest.mark.parametrize("n", [2, 3, 63, 64, 65, 130])
@pytest.mark.parametrize("shape", [1, 2])
def test_beams_smaller_than_a_few_wavefronts(lib, n, shape):
    assert _run(lib, n, (8, 8, 8), shape, 8) < TOL


def test_largest_grid_along_one_axis(lib):
    # 256 nodes: the padded transform along x has 512 points, the plan's limit
    assert _run(lib, 20_000, (256, 8, 12), 2, 6) < TOL


def test_radix3_grid(lib):
    # 2n = 96 = 2^5 3, 72 = 2^3 3^2, 54 = 2 3^3
    assert _run(lib, 12_000, (48, 36, 27), 1, 6) < TOL


def test_largest_tile_count(lib):
    # 4096 tiles of 2 x 2 x 4 nodes on a 32^3 grid
    assert _run(lib, 30_000, (32, 32, 32), 2, 6,
                tuning={"tile": (2, 2, 4), "chunk": 2048}) < TOL


def test_zero_extent_along_one_axis_is_an_error(lib):
    cfg = workloads.SMALL
    n = 1000
    xi = workloads.draw_xi(cfg, n=n)
    xi[2] = 0.0                      # y = 0 for every particle: no grid spacing along y
    xi[3] = 0.0
    b = lib.Beam(n, cfg.qm_qeeV, cfg.charge_C, cfg.kin_energy_MeV, cfg.mass_MeV, 1, (8, 8, 8))
    sig = np.array(cfg.sigma_matrix)
    b.init_from_normals(sig, torch.from_numpy(xi).cuda())
    b.deposit()
    assert b.check() == lib.PIC_EDOMAIN


@pytest.mark.parametrize("grid_fp32", [False, True])
def test_misaligned_grid_pointers_are_rejected(lib, grid_fp32):
    # a grid or particle-field pointer off its element's alignment is an argument error,
    # reported before anything is enqueued
    cfg = workloads.SMALL
    b = lib.Beam(1000, cfg.qm_qeeV, cfg.charge_C, cfg.kin_energy_MeV, cfg.mass_MeV, 1,
                 (8, 8, 8), grid_fp32=grid_fp32)
    b.init(cfg.sigma_matrix, seed=1)
    es = 4 if grid_fp32 else 8
    raw = torch.zeros(3 * 8 ** 3 * es + 64, dtype=torch.uint8, device="cuda")
    off = raw.data_ptr() + (es // 2)      # inside the buffer, off the element boundary
    good = b.new_E()
    rho = b.new_rho()
    assert lib._lib.pic_deposit(b._h, lib.ctypes.c_void_p(off), lib._stream()) == lib.PIC_EINVAL
    assert lib._lib.pic_poisson_solve(b._h, lib.ctypes.c_void_p(off), None,
                                      lib._ptr(good), lib._stream()) == lib.PIC_EINVAL
    assert lib._lib.pic_gather(b._h, lib._ptr(good), lib.ctypes.c_void_p(off),
                               lib._stream()) == lib.PIC_EINVAL
    assert lib._lib.pic_push(b._h, lib.PUSH_KICK, 0.1, lib.ctypes.c_void_p(off),
                             lib._stream()) == lib.PIC_EINVAL
    # the aligned calls still work, and nothing was flagged
    b.deposit(rho)
    assert b.check() == lib.PIC_OK
    b.close()
