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
}
