// Antiderivative of 1/r used by the integrated Green's function (see igf.hip).
#pragma once
#include "ddmath.hpp"

namespace pic {

// corner coordinate e_m = 0 (m = 0) or (m - 1/2) h, exact as a double pair
PIC_HD __forceinline__ ddv corner_coord(int m, double h) {
  if (m == 0) return {0.0, 0.0};
  return two_prod((double)m - 0.5, h);
}

PIC_HD inline ddv antiderivative(ddv x, ddv y, ddv z) {
  const bool x0 = x.hi == 0.0, y0 = y.hi == 0.0, z0 = z.hi == 0.0;
  ddv x2 = dd_mul(x, x), y2 = dd_mul(y, y), z2 = dd_mul(z, z);
  ddv r = dd_sqrt(dd_add(dd_add(x2, y2), z2));
  ddv xy = dd_mul(x, y), yz = dd_mul(y, z), zx = dd_mul(z, x);
  ddv zero = {0.0, 0.0};
  ddv t1 = (x0 || y0) ? zero : dd_mul(xy, dd_log(dd_add(z, r)));
  ddv t2 = (y0 || z0) ? zero : dd_mul(yz, dd_log(dd_add(x, r)));
  ddv t3 = (z0 || x0) ? zero : dd_mul(zx, dd_log(dd_add(y, r)));
  ddv t4 = x0 ? zero : dd_mul_d(dd_mul(x2, dd_atan(dd_div(yz, dd_mul(x, r)))), 0.5);
  ddv t5 = y0 ? zero : dd_mul_d(dd_mul(y2, dd_atan(dd_div(zx, dd_mul(y, r)))), 0.5);
  ddv t6 = z0 ? zero : dd_mul_d(dd_mul(z2, dd_atan(dd_div(xy, dd_mul(z, r)))), 0.5);
  return dd_sub(dd_add(dd_add(t1, t2), t3), dd_add(dd_add(t4, t5), t6));
}

}  // namespace pic
