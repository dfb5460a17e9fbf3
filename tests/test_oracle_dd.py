"""Pins of the oracle's double-double arithmetic against 50-digit mpmath."""
import mpmath as mp
import numpy as np
import pytest

from oracle import dd

mp.mp.dps = 50


def _points():
    rng = np.random.default_rng(11)
    x = rng.uniform(0.0, 1.0, 300) * 10.0 ** rng.integers(-12, 12, 300)
    x = np.concatenate([x, [1.0, 2.0, 0.5, np.sqrt(2.0), 1.0 / np.sqrt(2.0), 0.999999, 1.000001]])
    lo = x * rng.uniform(-1e-17, 1e-17, x.size)
    return x, lo


def _rel_err(res, ref):
    v = mp.mpf(float(res[0])) + mp.mpf(float(res[1]))
    return abs((v - ref) / ref) if ref != 0 else abs(v)


@pytest.mark.parametrize("name", ["log", "atan", "sqrt"])
def test_functions(name):
    x, lo = _points()
    f = getattr(dd, name)
    mf = getattr(mp, name)
    r = f((x, lo))
    worst = max(_rel_err((r[0][i], r[1][i]), mf(mp.mpf(float(x[i])) + mp.mpf(float(lo[i]))))
                for i in range(x.size))
    assert worst < 1e-30


def test_div_mul_add():
    rng = np.random.default_rng(3)
    a = (rng.uniform(-5, 5, 100), rng.uniform(-1e-16, 1e-16, 100))
    b = (rng.uniform(0.1, 7, 100), rng.uniform(-1e-17, 1e-17, 100))
    for op, mop in ((dd.div, lambda p, q: p / q), (dd.mul, lambda p, q: p * q),
                    (dd.add, lambda p, q: p + q), (dd.sub, lambda p, q: p - q)):
        r = op(a, b)
        for i in range(100):
            pa = mp.mpf(float(a[0][i])) + mp.mpf(float(a[1][i]))
            pb = mp.mpf(float(b[0][i])) + mp.mpf(float(b[1][i]))
            ref = mop(pa, pb)
            assert _rel_err((r[0][i], r[1][i]), ref) < 1e-30 or abs(ref) < 1e-30


def test_constants():
    assert abs(mp.mpf(dd.LN2[0]) + mp.mpf(dd.LN2[1]) - mp.log(2)) < 1e-32
    assert abs(mp.mpf(dd.PI_2[0]) + mp.mpf(dd.PI_2[1]) - mp.pi / 2) < 1e-32
