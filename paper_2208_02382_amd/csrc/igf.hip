// Integrated Green's function (Qiang et al., Phys. Rev. ST Accel. Beams 9, 044204, 2006):
// Gbar(i, j, k) = (1 / (hx hy hz)) * integral of dV/|r| over the rest-frame cell centred at
// (i hx, j hy, k hz), evaluated as the alternating 8-corner sum of the antiderivative
//   F(x,y,z) = xy ln(z+r) + yz ln(x+r) + zx ln(y+r)
//              - x^2/2 atan(yz/(xr)) - y^2/2 atan(zx/(yr)) - z^2/2 atan(xy/(zr)),
// terms with a zero prefactor being zero.  Cells on a coordinate plane (index 0) are folded onto
// [0, h/2] with weight 2 by the evenness of 1/r.
//
// The corner sum cancels by up to ~1e8 for far cells of elongated rest-frame cells (hz/hx of
// 80..8000 here), so F and the sum are carried in double-double arithmetic (ddmath.hpp) and
// the cell average is rounded to double once.
#include "igf_antideriv.hpp"
#include "internal.hpp"

namespace pic {

namespace {

// F at every corner (m_x, m_y, m_z), m_a = 0..n_a+1; corners[(mz (ny+2) + my)(nx+2) + mx]
__device__ __forceinline__ void igf_corners_body(const Geom* __restrict__ g, int nx, int ny, int nz,
                                                 double2* __restrict__ corners, int blk, int nblk) {
  if (g->status) return;
  const int cx = nx + 2, cy = ny + 2, cz = nz + 2;
  const int64_t total = (int64_t)cx * cy * cz;
  const double hx = g->h_rest[0], hy = g->h_rest[1], hz = g->h_rest[2];
  for (int64_t t = blk * 256ll + threadIdx.x; t < total; t += (int64_t)nblk * 256) {
    int mx = (int)(t % cx);
    int my = (int)((t / cx) % cy);
    int mz = (int)(t / ((int64_t)cx * cy));
    ddv f = antiderivative(corner_coord(mx, hx), corner_coord(my, hy), corner_coord(mz, hz));
    corners[t] = make_double2(f.hi, f.lo);
  }
}

__global__ __launch_bounds__(256) void k_igf_corners(const Geom* __restrict__ g, int nx, int ny,
                                                     int nz, double2* __restrict__ corners) {
  igf_corners_body(g, nx, ny, nz, corners, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(256) void k_igf_corners_batch(const BeamDev* __restrict__ beams) {
  const BeamDev& d = beams[blockIdx.y];
  igf_corners_body(d.geom, d.c.nx, d.c.ny, d.c.nz, d.corners, blockIdx.x, gridDim.x);
}

// Cell averages Gbar(i, j, k), i = 0..nx, j = 0..ny, k = 0..nz, from the corner values:
// successive double-double differences along x, then y, then z; cells on a coordinate plane
// carry weight 2 per folded axis; one division by the rest-frame cell volume; rounded to
// double once.  Output gd[(k (ny+1) + j)(nx+1) + i].
__device__ __forceinline__ void igf_cells_body(const Geom* __restrict__ g, int nx, int ny, int nz,
                                               const double2* __restrict__ corners,
                                               double* __restrict__ gd, int blk, int nblk) {
  if (g->status) return;
  const int cx = nx + 2, cy = ny + 2;
  const int ex = nx + 1, ey = ny + 1;
  const int64_t total = (int64_t)ex * ey * (nz + 1);
  const double hx = g->h_rest[0], hy = g->h_rest[1], hz = g->h_rest[2];
  const ddv vol = dd_mul_d(two_prod(hx, hy), hz);
  for (int64_t t = blk * 256ll + threadIdx.x; t < total; t += (int64_t)nblk * 256) {
    const int i = (int)(t % ex);
    const int j = (int)((t / ex) % ey);
    const int k = (int)(t / ((int64_t)ex * ey));
    ddv dxy[2][2];
    for (int c = 0; c < 2; ++c)
      for (int b = 0; b < 2; ++b) {
        const int64_t base = ((int64_t)(k + c) * cy + (j + b)) * cx + i;
        const double2 f0 = corners[base], f1 = corners[base + 1];
        dxy[c][b] = dd_sub(ddv{f1.x, f1.y}, ddv{f0.x, f0.y});
      }
    ddv d = dd_sub(dd_sub(dxy[1][1], dxy[1][0]), dd_sub(dxy[0][1], dxy[0][0]));
    const double w = (i == 0 ? 2.0 : 1.0) * (j == 0 ? 2.0 : 1.0) * (k == 0 ? 2.0 : 1.0);
    d = {d.hi * w, d.lo * w};
    const ddv gbar = dd_div(d, vol);
    gd[t] = gbar.hi + gbar.lo;
  }
}

__global__ __launch_bounds__(256) void k_igf_cells(const Geom* __restrict__ g, int nx, int ny,
                                                   int nz, const double2* __restrict__ corners,
                                                   double* __restrict__ gd) {
  igf_cells_body(g, nx, ny, nz, corners, gd, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(256) void k_igf_cells_batch(const BeamDev* __restrict__ beams) {
  const BeamDev& d = beams[blockIdx.y];
  igf_cells_body(d.geom, d.c.nx, d.c.ny, d.c.nz, d.corners, d.Gd, blockIdx.x, gridDim.x);
}

// The field kernels' corner values: H_x, H_y, H_z at every corner, hc[a total + t] (double
// pairs), t = (mz (ny+2) + my)(nx+2) + mx as for F.
__global__ __launch_bounds__(256) void k_igf_field_corners(const Geom* __restrict__ g, int nx,
                                                           int ny, int nz,
                                                           double2* __restrict__ hc) {
  if (g->status) return;
  const int cx = nx + 2, cy = ny + 2, cz = nz + 2;
  const int64_t total = (int64_t)cx * cy * cz;
  const double hx = g->h_rest[0], hy = g->h_rest[1], hz = g->h_rest[2];
  for (int64_t t = blockIdx.x * 256ll + threadIdx.x; t < total; t += (int64_t)gridDim.x * 256) {
    const int mx = (int)(t % cx);
    const int my = (int)((t / cx) % cy);
    const int mz = (int)(t / ((int64_t)cx * cy));
    ddv H[3];
    field_antiderivatives(corner_coord(mx, hx), corner_coord(my, hy), corner_coord(mz, hz), H);
    for (int a = 0; a < 3; ++a) hc[a * total + t] = make_double2(H[a].hi, H[a].lo);
  }
}

// Field kernels Kbar_a(i, j, k) = (1/V) integral over the cell of u_a/r^3 on the octant,
// gd3[a (nx+1)(ny+1)(nz+1) + (k (ny+1) + j)(nx+1) + i]: minus the 8-corner double-double sum
// of H_a; zero on the kernel's own zero plane (it is odd along a), weight 2 per other axis
// whose index is 0 (even there, folded); one division by the cell volume, rounded once.
__global__ __launch_bounds__(256) void k_igf_field_cells(const Geom* __restrict__ g, int nx,
                                                         int ny, int nz,
                                                         const double2* __restrict__ hc,
                                                         double* __restrict__ gd3) {
  if (g->status) return;
  const int cx = nx + 2, cy = ny + 2;
  const int ex = nx + 1, ey = ny + 1;
  const int64_t ctotal = (int64_t)cx * cy * (nz + 2);
  const int64_t total = (int64_t)ex * ey * (nz + 1);
  const double hx = g->h_rest[0], hy = g->h_rest[1], hz = g->h_rest[2];
  const ddv vol = dd_mul_d(two_prod(hx, hy), hz);
  for (int64_t t = blockIdx.x * 256ll + threadIdx.x; t < total; t += (int64_t)gridDim.x * 256) {
    const int i = (int)(t % ex);
    const int j = (int)((t / ex) % ey);
    const int k = (int)(t / ((int64_t)ex * ey));
    const int idx[3] = {i, j, k};
    for (int a = 0; a < 3; ++a) {
      double w = idx[a] == 0 ? 0.0 : -1.0;
      for (int b = 0; b < 3; ++b)
        if (b != a && idx[b] == 0) w *= 2.0;
      double out = 0.0;
      if (w != 0.0) {
        const double2* h = hc + a * ctotal;
        ddv dxy[2][2];
        for (int c = 0; c < 2; ++c)
          for (int b = 0; b < 2; ++b) {
            const int64_t base = ((int64_t)(k + c) * cy + (j + b)) * cx + i;
            const double2 f0 = h[base], f1 = h[base + 1];
            dxy[c][b] = dd_sub(ddv{f1.x, f1.y}, ddv{f0.x, f0.y});
          }
        ddv d = dd_sub(dd_sub(dxy[1][1], dxy[1][0]), dd_sub(dxy[0][1], dxy[0][0]));
        d = {d.hi * w, d.lo * w};
        const ddv kbar = dd_div(d, vol);
        out = kbar.hi + kbar.lo;
      }
      gd3[a * total + t] = out;
    }
  }
}

// Corner values of the kernels' h-derivatives (dh_corner_functions): nf = 3 (potential) or 9
// (field) double pairs per corner, dc[f ctotal + t], t as for F.
template <bool FIELD>
__global__ __launch_bounds__(256) void k_igf_dh_corners(const Geom* __restrict__ g, int nx,
                                                        int ny, int nz,
                                                        double2* __restrict__ dc) {
  if (g->status) return;
  constexpr int NF = FIELD ? 9 : 3;
  const int cx = nx + 2, cy = ny + 2, cz = nz + 2;
  const int64_t total = (int64_t)cx * cy * cz;
  const double hx = g->h_rest[0], hy = g->h_rest[1], hz = g->h_rest[2];
  for (int64_t t = blockIdx.x * 256ll + threadIdx.x; t < total; t += (int64_t)gridDim.x * 256) {
    const int mx = (int)(t % cx);
    const int my = (int)((t / cx) % cy);
    const int mz = (int)(t / ((int64_t)cx * cy));
    ddv v[NF];
    dh_corner_functions<FIELD>(corner_coord(mx, hx), corner_coord(my, hy), corner_coord(mz, hz),
                               v);
    for (int f = 0; f < NF; ++f) dc[f * total + t] = make_double2(v[f].hi, v[f].lo);
  }
}

// The derivative kernels on the octant: gd[f total + (k (ny+1) + j)(nx+1) + i] =
// d kernel_f / d h_b (b = f for the potential, f % 3 for the field) from the corner values
template <bool FIELD>
__global__ __launch_bounds__(256) void k_igf_dh_cells(const Geom* __restrict__ g, int nx, int ny,
                                                      int nz, const double2* __restrict__ dc,
                                                      double* __restrict__ gd) {
  if (g->status) return;
  constexpr int NF = FIELD ? 9 : 3;
  const int cx = nx + 2, cy = ny + 2;
  const int ex = nx + 1, ey = ny + 1;
  const int64_t ctotal = (int64_t)cx * cy * (nz + 2);
  const int64_t total = (int64_t)ex * ey * (nz + 1);
  const double h[3] = {g->h_rest[0], g->h_rest[1], g->h_rest[2]};
  const ddv vol = dd_mul_d(two_prod(h[0], h[1]), h[2]);
  for (int64_t t = blockIdx.x * 256ll + threadIdx.x; t < total; t += (int64_t)gridDim.x * 256) {
    const int i = (int)(t % ex);
    const int j = (int)((t / ex) % ey);
    const int k = (int)(t / ((int64_t)ex * ey));
    for (int f = 0; f < NF; ++f) {
      const double2* src = dc + f * ctotal;
      ddv c[8];
      for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
          for (int dx = 0; dx < 2; ++dx) {
            const double2 v = src[((int64_t)(k + dz) * cy + (j + dy)) * cx + i + dx];
            c[(dz * 2 + dy) * 2 + dx] = ddv{v.x, v.y};
          }
      const int b = FIELD ? f % 3 : f;
      gd[f * total + t] = dh_cell_value(c, dh_fold(FIELD, f, i, j, k), dd_mul_d(vol, h[b]));
    }
  }
}

int grid_for(int64_t total) {
  int64_t b = (total + 255) / 256;
  if (b > 16384) b = 16384;
  return (int)(b < 1 ? 1 : b);
}

}  // namespace

hipError_t launch_igf_corners(const Geom* g, int nx, int ny, int nz, double2* corners,
                              hipStream_t s) {
  int64_t total = (int64_t)(nx + 2) * (ny + 2) * (nz + 2);
  hipLaunchKernelGGL(k_igf_corners, dim3(grid_for(total)), dim3(256), 0, s, g, nx, ny, nz,
                     corners);
  return hipGetLastError();
}

hipError_t launch_igf_cells(const Geom* g, int nx, int ny, int nz, const double2* corners,
                            double* gd, hipStream_t s) {
  int64_t total = (int64_t)(nx + 1) * (ny + 1) * (nz + 1);
  hipLaunchKernelGGL(k_igf_cells, dim3(grid_for(total)), dim3(256), 0, s, g, nx, ny, nz, corners,
                     gd);
  return hipGetLastError();
}

hipError_t launch_igf_field(const Geom* g, int nx, int ny, int nz, double2* hc, double* gd3,
                            hipStream_t s) {
  const int64_t corners = (int64_t)(nx + 2) * (ny + 2) * (nz + 2);
  hipLaunchKernelGGL(k_igf_field_corners, dim3(grid_for(corners)), dim3(256), 0, s, g, nx, ny,
                     nz, hc);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t cells = (int64_t)(nx + 1) * (ny + 1) * (nz + 1);
  hipLaunchKernelGGL(k_igf_field_cells, dim3(grid_for(cells)), dim3(256), 0, s, g, nx, ny, nz, hc,
                     gd3);
  return hipGetLastError();
}

hipError_t launch_igf_dh(const Geom* g, int nx, int ny, int nz, bool field, double2* dc,
                         double* gd, hipStream_t s) {
  const int64_t corners = (int64_t)(nx + 2) * (ny + 2) * (nz + 2);
  const int64_t cells = (int64_t)(nx + 1) * (ny + 1) * (nz + 1);
  if (field) {
    hipLaunchKernelGGL(k_igf_dh_corners<true>, dim3(grid_for(corners)), dim3(256), 0, s, g, nx,
                       ny, nz, dc);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_igf_dh_cells<true>, dim3(grid_for(cells)), dim3(256), 0, s, g, nx, ny,
                       nz, dc, gd);
  } else {
    hipLaunchKernelGGL(k_igf_dh_corners<false>, dim3(grid_for(corners)), dim3(256), 0, s, g, nx,
                       ny, nz, dc);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_igf_dh_cells<false>, dim3(grid_for(cells)), dim3(256), 0, s, g, nx, ny,
                       nz, dc, gd);
  }
  return hipGetLastError();
}

hipError_t launch_batch_igf(const BeamDev* beams, int nb, int max_nx, int max_ny, int max_nz,
                            hipStream_t s) {
  const int64_t corners = (int64_t)(max_nx + 2) * (max_ny + 2) * (max_nz + 2);
  hipLaunchKernelGGL(k_igf_corners_batch, dim3(grid_for(corners), nb), dim3(256), 0, s, beams);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t cells = (int64_t)(max_nx + 1) * (max_ny + 1) * (max_nz + 1);
  hipLaunchKernelGGL(k_igf_cells_batch, dim3(grid_for(cells), nb), dim3(256), 0, s, beams);
  return hipGetLastError();
}

}  // namespace pic
