"""CPU unit tests of the kernels' double-double and integrated-Green's-function arithmetic
(ddmath.hpp, igf_antideriv.hpp built for the host as libpic_hostcheck.so), against 50-digit
mpmath and against the oracle."""
import ctypes
import os

import mpmath as mp
import numpy as np
import pytest

from oracle import igf

LIB = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_2208_02382_amd", "libpic_hostcheck.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="host check library not built")


@pytest.fixture(scope="module")
def lib():
    return ctypes.CDLL(LIB)


@pytest.mark.parametrize("fn,name", [(0, "log"), (1, "atan"), (2, "sqrt")])
def test_dd_functions(lib, fn, name):
    mp.mp.dps = 50
    rng = np.random.default_rng(5)
    x = rng.uniform(0, 1, 200) * 10.0 ** rng.integers(-8, 8, 200)
    lo = x * rng.uniform(-1e-17, 1e-17, 200)
    inp = np.ascontiguousarray(np.stack([x, lo], 1).ravel())
    out = np.zeros_like(inp)
    lib.pic_hostcheck_dd(fn, 200, inp.ctypes.data_as(ctypes.c_void_p),
                         out.ctypes.data_as(ctypes.c_void_p))
    f = getattr(mp, name)
    worst = max(abs((mp.mpf(out[2 * i]) + mp.mpf(out[2 * i + 1])
                     - f(mp.mpf(x[i]) + mp.mpf(lo[i]))) / f(mp.mpf(x[i]) + mp.mpf(lo[i])))
                for i in range(200))
    assert worst < 1e-30


def test_dd_atan2(lib):
    # atan(p/q) without forming p/q (the corner functions' arctangents), over ratios from 0 to
    # 1e8, at and next to 1 (where the inverse branch takes over), against 50-digit mpmath
    mp.mp.dps = 50
    rng = np.random.default_rng(6)
    m = 300
    ratio = np.concatenate([rng.uniform(0, 1, 100) * 10.0 ** rng.integers(-8, 8, 100),
                            1.0 + rng.uniform(-1e-15, 1e-15, 100),
                            rng.uniform(0.0, 2.0, 98), [0.0, 1.0]])
    q = rng.uniform(1e-4, 10.0, m)
    p = ratio * q
    plo = p * rng.uniform(-1e-17, 1e-17, m)
    qlo = q * rng.uniform(-1e-17, 1e-17, m)
    inp = np.ascontiguousarray(np.stack([p, plo, q, qlo], 1).ravel())
    out = np.zeros(2 * m)
    lib.pic_hostcheck_dd_atan2(m, inp.ctypes.data_as(ctypes.c_void_p),
                               out.ctypes.data_as(ctypes.c_void_p))
    worst = 0.0
    for i in range(m):
        ref = mp.atan((mp.mpf(p[i]) + mp.mpf(plo[i])) / (mp.mpf(q[i]) + mp.mpf(qlo[i])))
        got = mp.mpf(out[2 * i]) + mp.mpf(out[2 * i + 1])
        err = abs(got - ref) if ref == 0 else abs((got - ref) / ref)
        worst = max(worst, err)
    assert worst < 1e-30


@pytest.mark.parametrize("h", [(1.0, 1.0, 1.0), (1.0, 1.0, 80.0), (3e-4, 3.1e-4, 2.5e-2),
                               (1e-4, 1e-4, 0.78)])
def test_kernel_igf_equals_oracle(lib, h):
    n = 20
    g = np.zeros((n + 1) ** 3)
    lib.pic_hostcheck_igf(n, n, n, ctypes.c_double(h[0]), ctypes.c_double(h[1]),
                          ctypes.c_double(h[2]), g.ctypes.data_as(ctypes.c_void_p))
    go = igf.cell_average(n, n, n, *h)
    # both are the cell average rounded once from a double-double value
    assert np.abs(g.reshape(go.shape) - go).max() <= 2.3e-16 * np.abs(go).max()
    assert (np.abs(g.reshape(go.shape) - go) / np.abs(go)).max() < 2.3e-16


def test_dd_tables_match_their_generator():
    import subprocess
    import sys
    d = os.path.join(os.path.dirname(LIB), "csrc")
    out = subprocess.run([sys.executable, os.path.join(d, "gen_dd_tables.py")], check=True,
                         capture_output=True, text=True).stdout
    assert out == open(os.path.join(d, "dd_tables.hpp")).read()


@pytest.mark.parametrize("h", [(1.0, 1.0, 1.0), (3e-4, 3.1e-4, 2.5e-2), (1e-4, 1e-4, 0.78)])
@pytest.mark.parametrize("field", [0, 1])
def test_kernel_h_derivatives_equal_oracle(lib, h, field):
    # the device's corner functions of the kernels' h-derivatives (reduced forms of
    # r_b H_b - F and r_b B_ab + H_a) and their folded cell sums, against the oracle's
    # unreduced double-double forms: both are rounded once from a double-double value
    nx, ny, nz = 9, 7, 8
    nf = 9 if field else 3
    cells = (nx + 1) * (ny + 1) * (nz + 1)
    out = np.zeros(nf * cells)
    lib.pic_hostcheck_igf_dh(field, nx, ny, nz, ctypes.c_double(h[0]), ctypes.c_double(h[1]),
                             ctypes.c_double(h[2]), out.ctypes.data_as(ctypes.c_void_p))
    for f in range(nf):
        if field:
            ref = igf.field_cell_average_dh(nx, ny, nz, *h, f // 3, f % 3)
        else:
            ref = igf.cell_average_dh(nx, ny, nz, *h, f)
        got = out[f * cells:(f + 1) * cells].reshape(ref.shape)
        assert np.abs(got - ref).max() <= 4.5e-16 * np.abs(ref).max(), f
