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

// The field's 2-D antiderivatives at a corner (x, y, z >= 0):
//   H_x = y L_z + z L_y - x A_x,  H_y = z L_x + x L_z - y A_y,  H_z = x L_y + y L_x - z A_z,
// L_u = ln(u + r), A_x = atan(y z/(x r)), A_y = atan(z x/(y r)), A_z = atan(x y/(z r)), every
// term with a zero prefactor taken as zero.  d^2 H_x / dy dz = 1/r (likewise for y and z), so
// the cell integral of x/r^3 = -d(1/r)/dx is minus the alternating 8-corner sum of H_x.  The
// logarithms and arctangents are those of F: three of each per corner.
PIC_HD inline void field_antiderivatives(ddv x, ddv y, ddv z, ddv H[3]) {
  const bool x0 = x.hi == 0.0, y0 = y.hi == 0.0, z0 = z.hi == 0.0;
  const ddv r = dd_sqrt(dd_add(dd_add(dd_mul(x, x), dd_mul(y, y)), dd_mul(z, z)));
  const ddv zero = {0.0, 0.0};
  // ln(u + r) is needed where one of the other two coordinates is non-zero, so r > 0 there
  const ddv Lx = (y0 && z0) ? zero : dd_log(dd_add(x, r));
  const ddv Ly = (z0 && x0) ? zero : dd_log(dd_add(y, r));
  const ddv Lz = (x0 && y0) ? zero : dd_log(dd_add(z, r));
  const ddv Ax = x0 ? zero : dd_atan(dd_div(dd_mul(y, z), dd_mul(x, r)));
  const ddv Ay = y0 ? zero : dd_atan(dd_div(dd_mul(z, x), dd_mul(y, r)));
  const ddv Az = z0 ? zero : dd_atan(dd_div(dd_mul(x, y), dd_mul(z, r)));
  H[0] = dd_sub(dd_add(y0 ? zero : dd_mul(y, Lz), z0 ? zero : dd_mul(z, Ly)),
                x0 ? zero : dd_mul(x, Ax));
  H[1] = dd_sub(dd_add(z0 ? zero : dd_mul(z, Lx), x0 ? zero : dd_mul(x, Lz)),
                y0 ? zero : dd_mul(y, Ay));
  H[2] = dd_sub(dd_add(x0 ? zero : dd_mul(x, Ly), y0 ? zero : dd_mul(y, Lx)),
                z0 ? zero : dd_mul(z, Az));
}

}  // namespace pic
