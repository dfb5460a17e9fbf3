"""Pins of the oracle's Philox4x32-10 generator.

Known-answer vectors of Philox4x32 with 10 rounds from the Random123 distribution of Salmon et
al. (SC'11): (counter, key) -> output, all words hexadecimal.
"""
import numpy as np

from oracle import rng

KAT = [
    ((0x00000000, 0x00000000, 0x00000000, 0x00000000), (0x00000000, 0x00000000),
     (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)),
    ((0xffffffff, 0xffffffff, 0xffffffff, 0xffffffff), (0xffffffff, 0xffffffff),
     (0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)),
    ((0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344), (0xa4093822, 0x299f31d0),
     (0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1)),
]


def test_philox_kat():
    for ctr, key, out in KAT:
        got = rng.philox4x32_10(np.array(ctr, dtype=np.uint64).reshape(4, 1), key)[:, 0]
        assert tuple(int(v) for v in got) == out


def test_uniform_range_and_beam_statistics():
    n = 200_000
    xi = rng.beam_xi(n, seed=12345, n_halo=0)
    # standard normal rows: mean 0, variance 1, uncorrelated (5 / sqrt(n) bounds)
    tol = 5.0 / np.sqrt(n)
    assert np.all(np.abs(xi.mean(axis=1)) < tol)
    c = np.cov(xi)
    assert np.all(np.abs(np.diag(c) - 1.0) < 2 * tol * np.sqrt(2))
    assert np.all(np.abs(c - np.diag(np.diag(c))) < tol)
    w = rng.philox4x32_10(np.stack([np.arange(1000, dtype=np.uint64)] + [np.zeros(1000, np.uint64)] * 3), (7, 0))
    ua, ub = rng.uniforms(w)
    assert ua.min() > 0 and ua.max() <= 1 and ub.min() > 0 and ub.max() <= 1


def test_halo_rows_uniform():
    n = 10_000
    xi = rng.beam_xi(n, seed=9, n_halo=1000)
    h = xi[:, -1000:]
    assert h.min() > -4.0 and h.max() <= 4.0
    assert abs(h.var() - 64.0 / 12.0) < 0.3


def test_waterbag_draws_fill_the_ball_uniformly():
    # uniform in the 6-ball of radius R = sqrt(8): |xi| <= R, (|xi|/R)^6 ~ U(0, 1) (the radial
    # law of a uniform ball), isotropic, unit covariance
    n = 100_000
    xi = rng.waterbag_xi(n, seed=777)
    r = np.sqrt(np.sum(xi * xi, axis=0))
    R = np.sqrt(8.0)
    assert r.max() <= R * (1 + 1e-15)
    v = np.sort((r / R) ** 6)
    ks = np.max(np.maximum(np.arange(1, n + 1) / n - v, v - np.arange(n) / n))
    assert ks < 1.63 / np.sqrt(n)   # Kolmogorov-Smirnov, 1 % level
    tol = 5.0 / np.sqrt(n)
    assert np.all(np.abs(xi.mean(axis=1)) < tol)
    c = np.cov(xi)
    assert np.all(np.abs(np.diag(c) - 1.0) < 3 * tol)
    assert np.all(np.abs(c - np.diag(np.diag(c))) < tol)
    # half the radius holds 1/64 of a uniform 6-ball
    assert abs(np.mean(r < R / 2) - 1 / 64) < 5 * np.sqrt(1 / 64 / n)
    # the directions are those of the Gaussian draws of the same counters
    g = rng.beam_xi(n, seed=777, n_halo=0)
    cos = np.sum(g * xi, axis=0) / (np.sqrt(np.sum(g * g, axis=0)) * r)
    assert np.all(np.abs(cos - 1.0) < 1e-12)
