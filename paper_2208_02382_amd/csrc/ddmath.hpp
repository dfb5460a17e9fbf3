// Double-double arithmetic on the device.
//
// A value is an unevaluated sum hi + lo of two doubles (about 106 bits).  Error-free
// transformations: Knuth's TwoSum and the FMA form of the exact product (a*b = p + fma(a,b,-p)).
// Elementary functions:
//   exp  -- k = round(t/ln2), r = t - k ln2 (ln2 as a double pair), exp(r) = (exp(r/512))^512
//           with a 14-term Taylor polynomial for exp(r/512) - 1 and nine squarings of 1 + e.
//   log  -- one Newton step on exp: y0 = log(a.hi) in double, log a = y0 + (a exp(-y0) - 1)
//           - (a exp(-y0) - 1)^2/2 (the correction is ~1e-16, so two terms suffice).
//   atan -- a > 1 uses pi/2 - atan(1/a); three halvings t -> t/(1 + sqrt(1 + t^2)) bring the
//           argument below tan(pi/32); then the alternating Taylor series (18 terms).
//   sqrt -- Karp-Markstein: one correction of the double reciprocal square root.
// No fast-math and no contraction: TwoSum and FastTwoSum are exact only if every + and - is
// rounded on its own.  hipcc contracts a*b + c into an fma by default in device code, which
// silently turns these sequences into plain double arithmetic, so contraction is switched off
// for every translation unit that includes this header (and igf.hip is also built with
// -ffp-contract=off).  The only fused multiply-adds are the explicit std::fma calls.
#pragma once
#pragma clang fp contract(off)
#include <hip/hip_runtime.h>
#include <cmath>

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

PIC_HD __forceinline__ ddv dd_div(ddv a, ddv b) {
  double q1 = a.hi / b.hi;
  ddv r = dd_sub(a, dd_mul_d(b, q1));
  double q2 = r.hi / b.hi;
  r = dd_sub(r, dd_mul_d(b, q2));
  double q3 = r.hi / b.hi;
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

// 1/(k+1)! for k = 0..13 as double pairs (hi = nearest double, lo = remainder).
constexpr double kInvFact[14][2] = {
    {1.0, 0.0},
    {0.5, 0.0},
    {0.16666666666666666, 9.25185853854297e-18},
    {0.041666666666666664, 2.3129646346357427e-18},
    {0.008333333333333333, 1.1564823173178714e-19},
    {0.001388888888888889, -5.300543954373577e-20},
    {0.0001984126984126984, 1.7209558293420705e-22},
    {2.48015873015873e-05, 2.1511947866775882e-23},
    {2.7557319223985893e-06, -1.858393274046472e-22},
    {2.755731922398589e-07, 2.3767714622250297e-23},
    {2.505210838544172e-08, -1.448814070935912e-24},
    {2.08767569878681e-09, -1.20734505911326e-25},
    {1.6059043836821613e-10, 1.2585294588752098e-26},
    {1.1470745597729725e-11, 2.0655512752830745e-28},
};

// 1/(2k+1) for k = 0..17 as double pairs.
constexpr double kInvOdd[18][2] = {
    {1.0, 0.0},
    {0.3333333333333333, 1.850371707708594e-17},
    {0.2, -1.1102230246251566e-17},
    {0.14285714285714285, 7.93016446160826e-18},
    {0.1111111111111111, 6.1679056923619804e-18},
    {0.09090909090909091, -2.523234146875356e-18},
    {0.07692307692307693, -4.270088556250602e-18},
    {0.06666666666666667, 9.251858538542971e-19},
    {0.058823529411764705, 8.163404592832033e-19},
    {0.05263157894736842, 2.921639538487254e-18},
    {0.047619047619047616, 2.64338815386942e-18},
    {0.043478260869565216, 1.206764157201257e-18},
    {0.04, -8.326672684688674e-19},
    {0.037037037037037035, 2.05596856412066e-18},
    {0.034482758620689655, 4.785444071660157e-19},
    {0.03225806451612903, 8.953411488912552e-19},
    {0.030303030303030304, -8.410780489584519e-19},
    {0.02857142857142857, 8.921435019309293e-19},
};

// exp of a double argument t, |t| < 700, to double-double accuracy.
PIC_HD inline ddv dd_exp_d(double t) {
  double k = std::rint(t * 1.4426950408889634);   // t / ln 2
  // r = t - k ln2; k*kLn2Hi and k*kLn2Lo are formed exactly with two_prod
  ddv r = dd_sub(dd_make(t), dd_add(two_prod(k, kLn2Hi), two_prod(k, kLn2Lo)));
  ddv s = {std::ldexp(r.hi, -9), std::ldexp(r.lo, -9)};      // |s| < 6.8e-4
  // e = exp(s) - 1 = s (1/1! + s (1/2! + ... + s/14!)); truncation error < 1e-50
  ddv e = {kInvFact[13][0], kInvFact[13][1]};
  for (int q = 12; q >= 0; --q) e = dd_add(dd_mul(e, s), ddv{kInvFact[q][0], kInvFact[q][1]});
  e = dd_mul(e, s);
  // (1 + e)^512 by nine squarings, kept as e: (1 + e)^2 - 1 = 2e + e^2
  for (int q = 0; q < 9; ++q) e = dd_add(dd_mul_d(e, 2.0), dd_mul(e, e));
  ddv res = dd_add(dd_make(1.0), e);
  int ki = (int)k;
  return {std::ldexp(res.hi, ki), std::ldexp(res.lo, ki)};
}

// natural log of a positive double-double.
PIC_HD inline ddv dd_log(ddv a) {
  double y0 = std::log(a.hi);
  ddv ex = dd_exp_d(-y0);
  ddv u = dd_sub(dd_mul(a, ex), dd_make(1.0));   // ~1e-16
  // log(1+u) = u - u^2/2 + u^3/3: with |u| < 1e-15 the cubic term is below 1e-45
  ddv corr = dd_sub(u, dd_mul_d(dd_mul(u, u), 0.5));
  return dd_add(dd_make(y0), corr);
}

// arctangent of a non-negative double-double.
PIC_HD inline ddv dd_atan(ddv a) {
  bool inv = a.hi > 1.0;
  ddv t = inv ? dd_div(dd_make(1.0), a) : a;
  for (int q = 0; q < 3; ++q)
    t = dd_div(t, dd_add(dd_make(1.0), dd_sqrt(dd_add(dd_make(1.0), dd_mul(t, t)))));
  ddv t2 = dd_mul(t, t);
  // sum_{k=0}^{17} (-1)^k t^(2k) / (2k+1), Horner from the top term (k = 17 is odd)
  ddv p = dd_neg(ddv{kInvOdd[17][0], kInvOdd[17][1]});
  for (int k = 16; k >= 0; --k) {
    ddv ck = {kInvOdd[k][0], kInvOdd[k][1]};
    if (k & 1) ck = dd_neg(ck);
    p = dd_add(dd_mul(p, t2), ck);
  }
  ddv r = dd_mul_d(dd_mul(t, p), 8.0);
  if (inv) r = dd_sub(ddv{kPi2Hi, kPi2Lo}, r);
  return r;
}

}  // namespace pic
