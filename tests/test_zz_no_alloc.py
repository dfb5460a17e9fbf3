"""pic_moments_noalloc (the allocation-free form of pic_moments) against pic_moments, through the
C ABI, on two calls in a row, the second with a smaller input: the same kernels and reduction
shape, so the values must agree bit for bit."""
import ctypes

import numpy as np
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import paper_2208_02382_amd as p
    return p


def _unpack(out27):
    """(mean[6], cov[6][6]) from the 27-slot layout."""
    v = out27.cpu().numpy()
    cov = np.empty((6, 6))
    q = 6
    for a in range(6):
        for b in range(a, 6):
            cov[a, b] = cov[b, a] = v[q]
            q += 1
    return v[:6], cov


def _beam(lib, n, seed):
    cfg = workloads.MEDIUM
    b = lib.Beam(n, cfg.qm_qeeV, cfg.charge_C, cfg.kin_energy_MeV, cfg.mass_MeV, cfg.shape,
                 cfg.nodes)
    b.init(cfg.sigma_matrix, seed=seed, halo_frac=0.1)
    return b


def test_noalloc_moments_equal_pic_moments_on_two_calls(lib):
    big = _beam(lib, 300_001, 21)
    small = _beam(lib, 7_777, 22)
    # the allocation-free calls first, back to back on one stream, the second smaller
    out_big = torch.full((27,), float("nan"), dtype=torch.float64, device="cuda")
    out_small = torch.full((27,), float("nan"), dtype=torch.float64, device="cuda")
    lib.moments_noalloc(big.X, out_big)
    lib.moments_noalloc(small.X, out_small)
    torch.cuda.synchronize()
    for b, out in ((big, out_big), (small, out_small)):
        mean, cov = _unpack(out)
        m_ref, c_ref = b.moments()
        assert np.array_equal(mean, np.array(m_ref)), (b.n, mean, m_ref)
        assert np.array_equal(cov, np.array(c_ref)), b.n
    big.close()
    small.close()


def test_noalloc_moments_reject_bad_arguments(lib):
    X = torch.zeros((6, 16), dtype=torch.float64, device="cuda")
    out = torch.zeros(27, dtype=torch.float64, device="cuda")
    f = lib._lib.pic_moments_noalloc
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert f(ctypes.c_void_p(X.data_ptr()), 0, ctypes.c_void_p(out.data_ptr()), s) == lib.PIC_EINVAL
    assert f(ctypes.c_void_p(X.data_ptr()), 1 << 31, ctypes.c_void_p(out.data_ptr()), s) == \
        lib.PIC_EINVAL
    assert f(None, 16, ctypes.c_void_p(out.data_ptr()), s) == lib.PIC_EINVAL
    assert f(ctypes.c_void_p(X.data_ptr() + 4), 16, ctypes.c_void_p(out.data_ptr()), s) == \
        lib.PIC_EINVAL
    torch.cuda.synchronize()
    assert torch.all(out == 0)
