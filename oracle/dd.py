"""Double-double arithmetic on NumPy float64 arrays (oracle; test infrastructure).

A double-double value is a pair (hi, lo) of float64 arrays whose unevaluated sum carries about
106 bits.  The error-free transformations are the published ones: Knuth's TwoSum, Dekker's
splitting and exact product (Dekker, "A floating-point technique for extending the available
precision", Numer. Math. 18, 1971).  NumPy has no fused multiply-add, so the product uses
Dekker's split.  The elementary functions use textbook series with range reduction:

* log(a):  a = 2^e m with m in [1/sqrt2, sqrt2); log m = 2 atanh(s), s = (m-1)/(m+1),
           summed as s * sum_k s^(2k)/(2k+1).
* atan(a): atan(a) = pi/2 - atan(1/a) for a > 1, then three argument halvings
           t -> t / (1 + sqrt(1 + t^2)) (atan t = 2 atan of the halved argument), then the
           Taylor series of atan.
* sqrt(a): one Newton correction of the float64 square root (Karp and Markstein).

Pinned by tests/test_oracle_dd.py against mpmath at 50 digits.
"""
import numpy as np

_SPLIT = 134217729.0  # 2^27 + 1

# ln 2 and pi/2 split into a float64 pair; the test suite checks them against mpmath.
LN2 = (0.6931471805599453, 2.3190468138462996e-17)
PI_2 = (1.5707963267948966, 6.123233995736766e-17)


def two_sum(a, b):
    s = a + b
    bb = s - a
    err = (a - (s - bb)) + (b - bb)
    return s, err


def quick_two_sum(a, b):
    s = a + b
    err = b - (s - a)
    return s, err


def split(a):
    t = _SPLIT * a
    hi = t - (t - a)
    lo = a - hi
    return hi, lo


def two_prod(a, b):
    p = a * b
    ah, al = split(a)
    bh, bl = split(b)
    err = ((ah * bh - p) + ah * bl + al * bh) + al * bl
    return p, err


def dd(a):
    """Promote a float64 array to double-double."""
    a = np.asarray(a, dtype=np.float64)
    return a, np.zeros_like(a)


def add(a, b):
    s, e = two_sum(a[0], b[0])
    t, f = two_sum(a[1], b[1])
    e = e + t
    s, e = quick_two_sum(s, e)
    e = e + f
    return quick_two_sum(s, e)


def neg(a):
    return -a[0], -a[1]


def sub(a, b):
    return add(a, neg(b))


def mul(a, b):
    p, e = two_prod(a[0], b[0])
    e = e + (a[0] * b[1] + a[1] * b[0])
    return quick_two_sum(p, e)


def mul_d(a, b):
    """double-double times float64."""
    p, e = two_prod(a[0], b)
    e = e + a[1] * b
    return quick_two_sum(p, e)


def div(a, b):
    q1 = a[0] / b[0]
    r = sub(a, mul_d(b, q1))
    q2 = r[0] / b[0]
    r = sub(r, mul_d(b, q2))
    q3 = r[0] / b[0]
    q = quick_two_sum(q1, q2)
    return add(q, dd(q3))


def sqrt(a):
    """sqrt of a non-negative double-double; exact zero maps to zero."""
    hi = a[0]
    pos = hi > 0
    safe = np.where(pos, hi, 1.0)
    x = 1.0 / np.sqrt(safe)
    ax = safe * x
    ax_dd = dd(ax)
    a_safe = (np.where(pos, a[0], 1.0), np.where(pos, a[1], 0.0))
    r = sub(a_safe, mul(ax_dd, ax_dd))
    res = add(ax_dd, dd(r[0] * (x * 0.5)))
    return np.where(pos, res[0], 0.0), np.where(pos, res[1], 0.0)


def _recip_odd(k):
    """1/(2k+1) as a double-double scalar pair."""
    one = (np.float64(1.0), np.float64(0.0))
    return div(one, (np.float64(2 * k + 1), np.float64(0.0)))


_LOG_TERMS = 24     # s^2 <= 0.0295 -> 0.0295^24 < 1e-36
_ATAN_TERMS = 18    # t^2 <= 0.0097 -> 0.0097^18 < 1e-36
_LOG_C = [_recip_odd(k) for k in range(_LOG_TERMS)]
_ATAN_C = [_recip_odd(k) for k in range(_ATAN_TERMS)]


def log(a):
    """Natural log of a positive double-double."""
    hi = a[0]
    m, e = np.frexp(hi)               # hi = m 2^e, m in [0.5, 1)
    big = m < np.sqrt(0.5)
    e = np.where(big, e - 1, e)
    # scale a by 2^-e exactly (both parts)
    mm = (np.ldexp(a[0], -e), np.ldexp(a[1], -e))
    one = dd(np.ones_like(hi))
    s = div(sub(mm, one), add(mm, one))
    s2 = mul(s, s)
    p = (np.full_like(hi, _LOG_C[-1][0]), np.full_like(hi, _LOG_C[-1][1]))
    for k in range(_LOG_TERMS - 2, -1, -1):
        p = add(mul(p, s2), (np.full_like(hi, _LOG_C[k][0]), np.full_like(hi, _LOG_C[k][1])))
    logm = mul_d(mul(s, p), 2.0)
    ef = e.astype(np.float64)
    eln2 = mul_d((np.full_like(hi, LN2[0]), np.full_like(hi, LN2[1])), ef)
    return add(eln2, logm)


def atan(a):
    """Arctangent of a non-negative double-double."""
    hi = a[0]
    inv = hi > 1.0
    one = dd(np.ones_like(hi))
    safe = (np.where(hi > 0, a[0], 1.0), np.where(hi > 0, a[1], 0.0))
    t = div(one, safe)
    t = (np.where(inv, t[0], a[0]), np.where(inv, t[1], a[1]))
    for _ in range(3):
        t = div(t, add(one, sqrt(add(one, mul(t, t)))))
    t2 = mul(t, t)
    p = (np.full_like(hi, _ATAN_C[-1][0]), np.full_like(hi, _ATAN_C[-1][1]))
    if (_ATAN_TERMS - 1) % 2 == 1:
        p = neg(p)
    for k in range(_ATAN_TERMS - 2, -1, -1):
        c = (np.full_like(hi, _ATAN_C[k][0]), np.full_like(hi, _ATAN_C[k][1]))
        if k % 2 == 1:
            c = neg(c)
        p = add(mul(p, t2), c)
    r = mul_d(mul(t, p), 8.0)
    pi2 = (np.full_like(hi, PI_2[0]), np.full_like(hi, PI_2[1]))
    rinv = sub(pi2, r)
    return np.where(inv, rinv[0], r[0]), np.where(inv, rinv[1], r[1])


def to_float(a):
    return a[0] + a[1]
