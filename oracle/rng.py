"""Counter-based generator of the on-device beam initialisation (oracle; test infrastructure).

Philox4x32-10 as published by Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as easy
as 1, 2, 3", SC'11: ten rounds of the 4x32 Philox S-box with multipliers 0xD2511F53 and
0xCD9E8D57 and Weyl key increments 0x9E3779B9 and 0xBB67AE85.

Mapping of the generator to a beam (a reading of the library's own definition, so that both
sides can be compared draw by draw): particle i, draw block c in {0, 1, 2} uses counter
(i mod 2^32, i div 2^32, c, 0) and key (seed mod 2^32, seed div 2^32).  The four output words
(w0, w1, w2, w3) give two uniforms in (0, 1]:
    u_a = ((w0 >> 5) 2^26 + (w1 >> 6) + 1) 2^-53,  u_b = ((w2 >> 5) 2^26 + (w3 >> 6) + 1) 2^-53.
Core particles: Box-Muller, xi_{2c} = sqrt(-2 ln u_a) cos(2 pi u_b),
xi_{2c+1} = sqrt(-2 ln u_a) sin(2 pi u_b).  Halo particles: xi = -4 + 8 u.

Waterbag particles: the six Box-Muller normals g of draw blocks 0-2 give a direction, and
u_a of block 3 a radius: xi = sqrt(8) u_a^(1/6) g / |g|, uniform in the 6-ball of radius
sqrt(8) (Muller's method: an isotropic direction times a radius with CDF (r/R)^6).

Pinned by tests/test_oracle_rng.py (Random123 known-answer vectors for Philox4x32-10; the
radial law, bound and covariance of the Waterbag draws).
"""
import numpy as np

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint64(0x9E3779B9)
_W1 = np.uint64(0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def philox4x32_10(ctr, key):
    """ctr: uint array (4, n); key: (k0, k1).  Returns uint64 array (4, n) of 32-bit words."""
    c = [np.asarray(ctr[i], dtype=np.uint64) & _MASK for i in range(4)]
    k0 = np.uint64(key[0]) & _MASK
    k1 = np.uint64(key[1]) & _MASK
    for r in range(10):
        if r:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
        p0 = _M0 * c[0]
        p1 = _M1 * c[2]
        hi0, lo0 = p0 >> _S32, p0 & _MASK
        hi1, lo1 = p1 >> _S32, p1 & _MASK
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return np.stack(c)


def uniforms(words):
    """Two (0, 1] uniforms per 4-word block: rows (u_a, u_b)."""
    w = words.astype(np.uint64)
    a = ((w[0] >> np.uint64(5)) << np.uint64(26)) + (w[1] >> np.uint64(6)) + np.uint64(1)
    b = ((w[2] >> np.uint64(5)) << np.uint64(26)) + (w[3] >> np.uint64(6)) + np.uint64(1)
    scale = 2.0 ** -53
    return a.astype(np.float64) * scale, b.astype(np.float64) * scale


def beam_xi(n, seed, n_halo):
    """xi (6, n) as drawn by the on-device initialisation."""
    i = np.arange(n, dtype=np.uint64)
    key = (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    xi = np.empty((6, n))
    core = np.arange(n) < n - n_halo
    for c in range(3):
        ctr = np.stack([i & _MASK, i >> _S32, np.full(n, c, dtype=np.uint64),
                        np.zeros(n, dtype=np.uint64)])
        ua, ub = uniforms(philox4x32_10(ctr, key))
        rad = np.sqrt(-2.0 * np.log(ua))
        ang = 2.0 * np.pi * ub
        xi[2 * c] = np.where(core, rad * np.cos(ang), -4.0 + 8.0 * ua)
        xi[2 * c + 1] = np.where(core, rad * np.sin(ang), -4.0 + 8.0 * ub)
    return xi


def waterbag_xi(n, seed):
    """xi (6, n) of the on-device Waterbag initialisation: uniform in the ball of radius
    sqrt(8)."""
    i = np.arange(n, dtype=np.uint64)
    key = (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    g = np.empty((6, n))
    for c in range(3):
        ctr = np.stack([i & _MASK, i >> _S32, np.full(n, c, dtype=np.uint64),
                        np.zeros(n, dtype=np.uint64)])
        ua, ub = uniforms(philox4x32_10(ctr, key))
        rad = np.sqrt(-2.0 * np.log(ua))
        ang = 2.0 * np.pi * ub
        g[2 * c] = rad * np.cos(ang)
        g[2 * c + 1] = rad * np.sin(ang)
    ctr = np.stack([i & _MASK, i >> _S32, np.full(n, 3, dtype=np.uint64),
                    np.zeros(n, dtype=np.uint64)])
    ua, _ = uniforms(philox4x32_10(ctr, key))
    norm = np.sqrt(np.sum(g * g, axis=0))
    return np.sqrt(8.0) * np.power(ua, 1.0 / 6.0) * g / norm
