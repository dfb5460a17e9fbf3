// Double-double arithmetic on the device.
//
// A value is an unevaluated sum hi + lo of two doubles (about 106 bits).  Error-free
// transformations: Knuth's TwoSum and the FMA form of the exact product (a*b = p + fma(a,b,-p)).
// Elementary functions (table-driven argument reduction, then short series):
//   log  -- a = 2^e m, m in [1, 2); c = 1 + k/1024 nearest m; log a = e ln2 + log c
//           + 2 atanh(t), t = (m - c)/(m + c), |t| <= 1/4096, atanh by 5 series terms.
//   atan -- a > 1 uses pi/2 - atan(1/a); c = k/1024 nearest the argument x in [0, 1];
//           atan x = atan c + atan(t), t = (x - c)/(1 + x c), |t| <= 1/2048, 5 series terms.
//   sqrt -- Karp-Markstein: one correction of the double reciprocal square root.
// The tables log(1 + k/1024) and atan(k/1024) (dd_tables.hpp) are double pairs from 60-digit
// mpmath; series truncation errors are below 1e-33 relative.
// No fast-math and no contraction: TwoSum and FastTwoSum are exact only if every + and - is
// rounded on its own.  hipcc contracts a*b + c into an fma by default in device code, which
// silently turns these sequences into plain double arithmetic, so contraction is switched off
// for every translation unit that includes this header (and igf.hip is also built with
// -ffp-contract=off).  The only fused multiply-adds are the explicit std::fma calls.
#pragma once
#pragma clang fp contract(off)
#include <hip/hip_runtime.h>
#include <cmath>

#include "dd_tables.hpp"

// Callable from host code as well, so that the arithmetic can be unit-tested on a CPU.
#define PIC_HD __host__ __device__

namespace pic {

struct ddv {
  double hi, lo;
};

PIC_HD __forceinline__ ddv dd_make(double a) { return {a, 0.0}; }

PIC_HD __forceinline__ ddv two_sum(double a, double b) {
  double s = a + b;
  double bb = s - a;
  double e = (a - (s - bb)) + (b - bb);
  return {s, e};
}

PIC_HD __forceinline__ ddv fast_two_sum(double a, double b) {
  double s = a + b;
  double e = b - (s - a);
  return {s, e};
}

PIC_HD __forceinline__ ddv two_prod(double a, double b) {
  double p = a * b;
  return {p, std::fma(a, b, -p)};
}

PIC_HD __forceinline__ ddv dd_add(ddv a, ddv b) {
  ddv s = two_sum(a.hi, b.hi);
  ddv t = two_sum(a.lo, b.lo);
  s.lo += t.hi;
  s = fast_two_sum(s.hi, s.lo);
  s.lo += t.lo;
  return fast_two_sum(s.hi, s.lo);
}

PIC_HD __forceinline__ ddv dd_neg(ddv a) { return {-a.hi, -a.lo}; }
PIC_HD __forceinline__ ddv dd_sub(ddv a, ddv b) { return dd_add(a, dd_neg(b)); }

PIC_HD __forceinline__ ddv dd_mul(ddv a, ddv b) {
  ddv p = two_prod(a.hi, b.hi);
  p.lo = std::fma(a.hi, b.lo, std::fma(a.lo, b.hi, p.lo));
  return fast_two_sum(p.hi, p.lo);
}

PIC_HD __forceinline__ ddv dd_mul_d(ddv a, double b) {
  ddv p = two_prod(a.hi, b);
  p.lo = std::fma(a.lo, b, p.lo);
  return fast_two_sum(p.hi, p.lo);
}

// a / b: three partial quotients, each the current remainder times the double reciprocal of
// b.hi; the remainders are formed exactly (dd arithmetic), so each step removes the previous
// quotient's error whatever the reciprocal's rounding (one division instead of three).
PIC_HD __forceinline__ ddv dd_div(ddv a, ddv b) {
  const double rb = 1.0 / b.hi;
  double q1 = a.hi * rb;
  ddv r = dd_sub(a, dd_mul_d(b, q1));
  double q2 = r.hi * rb;
  r = dd_sub(r, dd_mul_d(b, q2));
  double q3 = r.hi * rb;
  return dd_add(fast_two_sum(q1, q2), dd_make(q3));
}

PIC_HD __forceinline__ ddv dd_sqrt(ddv a) {
  if (a.hi <= 0.0) return {0.0, 0.0};
  double x = 1.0 / std::sqrt(a.hi);
  double ax = a.hi * x;
  ddv d = dd_sub(a, two_prod(ax, ax));
  return two_sum(ax, d.hi * (x * 0.5));
}

// ln 2 and pi/2 as double pairs (hi = the double nearest the constant, lo = the remainder).
constexpr double kLn2Hi = 6.93147180559945286e-01;
constexpr double kLn2Lo = 2.31904681384629956e-17;
constexpr double kPi2Hi = 1.57079632679489656e+00;
constexpr double kPi2Lo = 6.12323399573676604e-17;

// 1/(2k+1) for k = 0..4 as double pairs.
constexpr double kInvOdd[5][2] = {
    {1.0, 0.0},
    {0.3333333333333333, 1.850371707708594e-17},
    {0.2, -1.1102230246251566e-17},
    {0.14285714285714285, 7.93016446160826e-18},
    {0.1111111111111111, 6.1679056923619804e-18},
};

// natural log of a positive double-double.
PIC_HD inline ddv dd_log(ddv a) {
  int e;
  std::frexp(a.hi, &e);  // a.hi = f 2^e, f in [1/2, 1)
  e -= 1;
  const ddv m = {std::ldexp(a.hi, -e), std::ldexp(a.lo, -e)};  // exact; m.hi in [1, 2)
  const int k = (int)std::rint((m.hi - 1.0) * 1024.0);         // 0..1024
  const double c = 1.0 + (double)k * 0.0009765625;
  const ddv t = dd_div(dd_sub(m, dd_make(c)), dd_add(m, dd_make(c)));
  const ddv t2 = dd_mul(t, t);
  // atanh t = t sum_{j=0}^{4} t^(2j)/(2j+1); the first omitted term is below 8e-38 t
  ddv p = {kInvOdd[4][0], kInvOdd[4][1]};
  for (int j = 3; j >= 0; --j) p = dd_add(dd_mul(p, t2), ddv{kInvOdd[j][0], kInvOdd[j][1]});
  const ddv at = dd_mul_d(dd_mul(t, p), 2.0);
  const ddv el2 = dd_add(two_prod((double)e, kLn2Hi), two_prod((double)e, kLn2Lo));
  return dd_add(dd_add(el2, ddv{kLogTab[k][0], kLogTab[k][1]}), at);
}

// arctangent of a non-negative double-double.
PIC_HD inline ddv dd_atan(ddv a) {
  const bool inv = a.hi > 1.0;
  const ddv x = inv ? dd_div(dd_make(1.0), a) : a;  // in [0, 1]
  const int k = (int)std::rint(x.hi * 1024.0);        // 0..1024
  const double c = (double)k * 0.0009765625;
  const ddv t = dd_div(dd_sub(x, dd_make(c)), dd_add(dd_make(1.0), dd_mul_d(x, c)));
  const ddv t2 = dd_mul(t, t);
  // atan t = t sum_{j=0}^{4} (-1)^j t^(2j)/(2j+1); the first omitted term is below 8e-35 t
  ddv p = ddv{kInvOdd[4][0], kInvOdd[4][1]};
  for (int j = 3; j >= 0; --j) {
    ddv cj = {kInvOdd[j][0], kInvOdd[j][1]};
    if (j & 1) cj = dd_neg(cj);
    p = dd_add(dd_mul(p, t2), cj);
  }
  ddv r = dd_add(ddv{kAtanTab[k][0], kAtanTab[k][1]}, dd_mul(t, p));
  if (inv) r = dd_sub(ddv{kPi2Hi, kPi2Lo}, r);
  return r;
}

// arctangent of p/q for double-doubles p >= 0, q > 0, without forming p/q: the ratio or its
// inverse, whichever is at most about 1, picks the table entry c = k/1024 from the leading
// parts, and atan(num/den) = atan c + atan(t) with t = (num - c den)/(den + c num), the same
// reduced argument as dd_atan's (x - c)/(1 + x c) for x = num/den, so one division serves both
// the ratio and the reduction.  The identity holds for any c >= 0, so a table entry chosen from
// rounded leading parts only widens |t| by a rounding error beyond 1/2048.
PIC_HD inline ddv dd_atan2(ddv p, ddv q) {
  const bool inv = p.hi > q.hi;
  const ddv num = inv ? q : p, den = inv ? p : q;
  const int k = (int)std::rint(num.hi / den.hi * 1024.0);  // 0..1024
  const double c = (double)k * 0.0009765625;
  const ddv t = dd_div(dd_sub(num, dd_mul_d(den, c)), dd_add(den, dd_mul_d(num, c)));
  const ddv t2 = dd_mul(t, t);
  ddv s = ddv{kInvOdd[4][0], kInvOdd[4][1]};
  for (int j = 3; j >= 0; --j) {
    ddv cj = {kInvOdd[j][0], kInvOdd[j][1]};
    if (j & 1) cj = dd_neg(cj);
    s = dd_add(dd_mul(s, t2), cj);
  }
  ddv r = dd_add(ddv{kAtanTab[k][0], kAtanTab[k][1]}, dd_mul(t, s));
  if (inv) r = dd_sub(ddv{kPi2Hi, kPi2Lo}, r);
  return r;
}

}  // namespace pic
