// Host build of the device arithmetic of the integrated Green's function (ddmath.hpp,
// igf_antideriv.hpp), exported for CPU unit tests of the kernels' math.  Not used by libpic.so.
#include "igf_antideriv.hpp"

extern "C" {

// double-double log / atan / sqrt of (hi, lo) pairs: in[2k], in[2k+1] -> out[2k], out[2k+1]
void pic_hostcheck_dd(int fn, int count, const double* in, double* out) {
  for (int k = 0; k < count; ++k) {
    pic::ddv a{in[2 * k], in[2 * k + 1]};
    pic::ddv r = fn == 0 ? pic::dd_log(a) : fn == 1 ? pic::dd_atan(a) : pic::dd_sqrt(a);
    out[2 * k] = r.hi;
    out[2 * k + 1] = r.lo;
  }
}

// double-double atan(p/q): in[4k..4k+3] = (p.hi, p.lo, q.hi, q.lo) -> out[2k], out[2k+1]
void pic_hostcheck_dd_atan2(int count, const double* in, double* out) {
  for (int k = 0; k < count; ++k) {
    pic::ddv r = pic::dd_atan2(pic::ddv{in[4 * k], in[4 * k + 1]},
                               pic::ddv{in[4 * k + 2], in[4 * k + 3]});
    out[2 * k] = r.hi;
    out[2 * k + 1] = r.lo;
  }
}

// Gbar(i, j, k) for i = 0..nx, j = 0..ny, k = 0..nz into out[((k (ny+1)) + j)(nx+1) + i],
// with the corner values and the 8-corner difference of the kernels.
void pic_hostcheck_igf(int nx, int ny, int nz, double hx, double hy, double hz, double* out) {
  const int cx = nx + 2, cy = ny + 2, cz = nz + 2;
  pic::ddv* F = new pic::ddv[(size_t)cx * cy * cz];
  for (int mz = 0; mz < cz; ++mz)
    for (int my = 0; my < cy; ++my)
      for (int mx = 0; mx < cx; ++mx)
        F[((size_t)mz * cy + my) * cx + mx] = pic::antiderivative(
            pic::corner_coord(mx, hx), pic::corner_coord(my, hy), pic::corner_coord(mz, hz));
  pic::ddv vol = pic::dd_mul_d(pic::two_prod(hx, hy), hz);
  for (int k = 0; k <= nz; ++k)
    for (int j = 0; j <= ny; ++j)
      for (int i = 0; i <= nx; ++i) {
        pic::ddv dxy[2][2];
        for (int c = 0; c < 2; ++c)
          for (int b = 0; b < 2; ++b) {
            size_t base = ((size_t)(k + c) * cy + (j + b)) * cx + i;
            dxy[c][b] = pic::dd_sub(F[base + 1], F[base]);
          }
        pic::ddv d = pic::dd_sub(pic::dd_sub(dxy[1][1], dxy[1][0]),
                                 pic::dd_sub(dxy[0][1], dxy[0][0]));
        double w = (i == 0 ? 2.0 : 1.0) * (j == 0 ? 2.0 : 1.0) * (k == 0 ? 2.0 : 1.0);
        d = {d.hi * w, d.lo * w};
        pic::ddv g = pic::dd_div(d, vol);
        out[((size_t)k * (ny + 1) + j) * (nx + 1) + i] = g.hi + g.lo;
      }
  delete[] F;
}

// The kernels' h-derivatives (field = 0: dGbar/dh_b, b = 0..2; field = 1: dKbar_a/dh_b,
// f = 3 a + b) on the octant, out[f cells + ((k (ny+1)) + j)(nx+1) + i], with the corner
// functions and cell sums of the kernels.
void pic_hostcheck_igf_dh(int field, int nx, int ny, int nz, double hx, double hy, double hz,
                          double* out) {
  const int nf = field ? 9 : 3;
  const int cx = nx + 2, cy = ny + 2, cz = nz + 2;
  const size_t ctotal = (size_t)cx * cy * cz;
  const size_t cells = (size_t)(nx + 1) * (ny + 1) * (nz + 1);
  pic::ddv* C = new pic::ddv[ctotal * nf];
  for (int mz = 0; mz < cz; ++mz)
    for (int my = 0; my < cy; ++my)
      for (int mx = 0; mx < cx; ++mx) {
        pic::ddv v[9];
        const pic::ddv x = pic::corner_coord(mx, hx), y = pic::corner_coord(my, hy),
                       z = pic::corner_coord(mz, hz);
        if (field)
          pic::dh_corner_functions<true>(x, y, z, v);
        else
          pic::dh_corner_functions<false>(x, y, z, v);
        for (int f = 0; f < nf; ++f) C[f * ctotal + ((size_t)mz * cy + my) * cx + mx] = v[f];
      }
  const double h[3] = {hx, hy, hz};
  const pic::ddv vol = pic::dd_mul_d(pic::two_prod(hx, hy), hz);
  for (int f = 0; f < nf; ++f)
    for (int k = 0; k <= nz; ++k)
      for (int j = 0; j <= ny; ++j)
        for (int i = 0; i <= nx; ++i) {
          pic::ddv c[8];
          for (int dz = 0; dz < 2; ++dz)
            for (int dy = 0; dy < 2; ++dy)
              for (int dx = 0; dx < 2; ++dx)
                c[(dz * 2 + dy) * 2 + dx] =
                    C[f * ctotal + ((size_t)(k + dz) * cy + (j + dy)) * cx + i + dx];
          const int b = field ? f % 3 : f;
          out[f * cells + ((size_t)k * (ny + 1) + j) * (nx + 1) + i] = pic::dh_cell_value(
              c, pic::dh_fold(field != 0, f, i, j, k), pic::dd_mul_d(vol, h[b]));
        }
  delete[] C;
}
}
