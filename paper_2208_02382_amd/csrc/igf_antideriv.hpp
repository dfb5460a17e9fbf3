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
  ddv t4 = x0 ? zero : dd_mul_d(dd_mul(x2, dd_atan2(yz, dd_mul(x, r))), 0.5);
  ddv t5 = y0 ? zero : dd_mul_d(dd_mul(y2, dd_atan2(zx, dd_mul(y, r))), 0.5);
  ddv t6 = z0 ? zero : dd_mul_d(dd_mul(z2, dd_atan2(xy, dd_mul(z, r))), 0.5);
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
  const ddv Ax = x0 ? zero : dd_atan2(dd_mul(y, z), dd_mul(x, r));
  const ddv Ay = y0 ? zero : dd_atan2(dd_mul(z, x), dd_mul(y, r));
  const ddv Az = z0 ? zero : dd_atan2(dd_mul(x, y), dd_mul(z, r));
  H[0] = dd_sub(dd_add(y0 ? zero : dd_mul(y, Lz), z0 ? zero : dd_mul(z, Ly)),
                x0 ? zero : dd_mul(x, Ax));
  H[1] = dd_sub(dd_add(z0 ? zero : dd_mul(z, Lx), x0 ? zero : dd_mul(x, Lz)),
                y0 ? zero : dd_mul(y, Ay));
  H[2] = dd_sub(dd_add(x0 ? zero : dd_mul(x, Ly), y0 ? zero : dd_mul(y, Lx)),
                z0 ? zero : dd_mul(z, Az));
}

// Corner functions of the kernels' derivatives in the rest-frame spacing h_b.  Substituting
// r = h s in the cell average gives d/dh_b avg(f) = (1/h_b) avg(r_b df/dr_b); integrating by
// parts in r_b turns that into an 8-corner sum of one corner function C, so
// d/dh_b avg(f) = fold / (V h_b) * (8-corner sum of C), folded as the kernel itself.
//   potential (f = 1/r):  C_b = r_b H_b - F, which reduces to
//     C_x = -y z L_x - x^2/2 A_x + y^2/2 A_y + z^2/2 A_z  (cyclic in x, y, z);
//   field (f = u_a/r^3):  C_ab = r_b B_ab + H_a with the face antiderivative B_aa =
//     atan(v w/(u_a r)) and B_ab = -ln(u_c + r) (c the third axis), which reduces to
//     C_xx = y L_z + z L_y, C_xy = z L_y - x A_x, C_xz = y L_z - x A_x, and cyclically.
// A term with a zero prefactor is zero (its logarithm or arctangent may be undefined there).
// out[b] for the potential (3 values), out[3 a + b] for the field (9 values).
template <bool FIELD>
PIC_HD inline void dh_corner_functions(ddv x, ddv y, ddv z, ddv* out) {
  const bool x0 = x.hi == 0.0, y0 = y.hi == 0.0, z0 = z.hi == 0.0;
  const ddv r = dd_sqrt(dd_add(dd_add(dd_mul(x, x), dd_mul(y, y)), dd_mul(z, z)));
  const ddv zero = {0.0, 0.0};
  const ddv Lx = (y0 && z0) ? zero : dd_log(dd_add(x, r));
  const ddv Ly = (z0 && x0) ? zero : dd_log(dd_add(y, r));
  const ddv Lz = (x0 && y0) ? zero : dd_log(dd_add(z, r));
  const ddv Ax = x0 ? zero : dd_atan2(dd_mul(y, z), dd_mul(x, r));
  const ddv Ay = y0 ? zero : dd_atan2(dd_mul(z, x), dd_mul(y, r));
  const ddv Az = z0 ? zero : dd_atan2(dd_mul(x, y), dd_mul(z, r));
  // coordinate times a logarithm / arctangent, zero with the coordinate
  auto cl = [&](ddv c, bool c0, ddv L) { return c0 ? zero : dd_mul(c, L); };
  if constexpr (!FIELD) {
    const ddv hx2 = dd_mul_d(dd_mul(x, x), 0.5), hy2 = dd_mul_d(dd_mul(y, y), 0.5),
              hz2 = dd_mul_d(dd_mul(z, z), 0.5);
    const ddv tx = x0 ? zero : dd_mul(hx2, Ax);
    const ddv ty = y0 ? zero : dd_mul(hy2, Ay);
    const ddv tz = z0 ? zero : dd_mul(hz2, Az);
    const ddv yzLx = (y0 || z0) ? zero : dd_mul(dd_mul(y, z), Lx);
    const ddv zxLy = (z0 || x0) ? zero : dd_mul(dd_mul(z, x), Ly);
    const ddv xyLz = (x0 || y0) ? zero : dd_mul(dd_mul(x, y), Lz);
    out[0] = dd_sub(dd_add(ty, tz), dd_add(yzLx, tx));
    out[1] = dd_sub(dd_add(tz, tx), dd_add(zxLy, ty));
    out[2] = dd_sub(dd_add(tx, ty), dd_add(xyLz, tz));
  } else {
    const ddv yLz = cl(y, y0, Lz), zLy = cl(z, z0, Ly), zLx = cl(z, z0, Lx);
    const ddv xLz = cl(x, x0, Lz), xLy = cl(x, x0, Ly), yLx = cl(y, y0, Lx);
    const ddv xAx = cl(x, x0, Ax), yAy = cl(y, y0, Ay), zAz = cl(z, z0, Az);
    out[0] = dd_add(yLz, zLy);  // (x, x)
    out[1] = dd_sub(zLy, xAx);  // (x, y)
    out[2] = dd_sub(yLz, xAx);  // (x, z)
    out[3] = dd_sub(zLx, yAy);  // (y, x)
    out[4] = dd_add(zLx, xLz);  // (y, y)
    out[5] = dd_sub(xLz, yAy);  // (y, z)
    out[6] = dd_sub(yLx, zAz);  // (z, x)
    out[7] = dd_sub(xLy, zAz);  // (z, y)
    out[8] = dd_add(xLy, yLx);  // (z, z)
  }
}

// fold / (V h_b) * (alternating 8-corner sum of c), c[(dz 2 + dy) 2 + dx] the corner values of
// one cell (d = 0 lower, 1 upper corner along each axis), rounded to double once; vhb = V h_b
PIC_HD inline double dh_cell_value(const ddv c[8], double fold, ddv vhb) {
  if (fold == 0.0) return 0.0;
  ddv dxy[2][2];
  for (int dz = 0; dz < 2; ++dz)
    for (int dy = 0; dy < 2; ++dy) dxy[dz][dy] = dd_sub(c[(dz * 2 + dy) * 2 + 1], c[(dz * 2 + dy) * 2]);
  ddv d = dd_sub(dd_sub(dxy[1][1], dxy[1][0]), dd_sub(dxy[0][1], dxy[0][0]));
  d = {d.hi * fold, d.lo * fold};
  const ddv v = dd_div(d, vhb);
  return v.hi + v.lo;
}

// folding weight of the octant cell (i, j, k) for derivative kernel f: the potential's are even
// along every axis (weight 2 per index-0 axis); the field's (a, b) = (f / 3, f % 3) are odd
// along a (zero on its index-0 plane) and even along the other two
PIC_HD inline double dh_fold(bool field, int f, int i, int j, int k) {
  const int idx[3] = {i, j, k};
  double w = 1.0;
  for (int q = 0; q < 3; ++q)
    if (idx[q] == 0) w *= (field && q == f / 3) ? 0.0 : 2.0;
  return w;
}

}  // namespace pic
