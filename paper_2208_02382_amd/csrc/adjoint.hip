// Reverse sweep (discrete adjoint) of the tracking loop.
//
// Gradients of J = w . (sigma_x, sigma_y, eps_x, eps_y) of the final beam with respect to the
// lattice elements' strengths, the initial coordinates and (given the draws xi of X0 = L xi)
// the Cholesky factor L.  Every step's grid geometry follows the particles (the box of the
// kick-point positions sets origin and spacing), and its terms are part of the gradient (below).
// Each linear operation is replaced by its transpose (apply_half_T for the half maps):
//   drift l          lam_px += l lam_x, lam_py += l lam_y, lam_delta += (l/gamma^2) lam_z
//   thin quad k      lam_x -= k lam_px, lam_y += k lam_py;  dJ/dk += sum(-x lam_px + y lam_py)
//   quadrupole half map M(k) per plane: lam <- M^T lam;  dJ/dk += sum lam_after . (dM/dk) x_before
//                    (the second half map's term from the state after it, as dM/dk M^-1 x_after)
//   kick over L      a_i = (C L lam_px, C L lam_py, gamma C L lam_delta)
//                    lam_r,i += sum_n grad W(r_i - r_n) (a_i . E'_n)            (k_adj_b, direct)
//                    e = sum_i W a_i (vector deposit, k_adj_a); psi = -sum_c D_c^T e_c on nodes
//                    -1..n (k_adj_div); chi = Gbar * psi / (4 pi eps0) on nodes 0..n-1
//                    (transposed solve, fft.hip); lam_r,i += q_m sum_n grad W(r_i - r_n) chi_n
//   geometry         with g_i the position gradient through the weights (the two terms above)
//                    and u_i = (r_i - origin)/h: dJ/dorigin_a = -sum g_i,a and
//                    dJ/dh_a = -sum g_i,a u_i,a (k_adj_b's block sums); dJ/dh'_b gets
//                    -sum_n e_b E'_b / h'_b (the centred difference) and
//                    sum_n Q_n (dGbar/dh'_b * psi)_n / (4 pi eps0) (the Green's function), or with
//                    the direct field sum_a sum_n e_a (dKbar_a/dh'_b * Q) / (4 pi eps0); h' is
//                    the rest-frame cell (h'_z = gamma h_z).  Through h = (max - min)/(n - 3.5)
//                    and origin = min - 1.25 h these go to the kick-point coordinate of the
//                    particle at the box's min (the first such index) and of the one at its
//                    max (k_adj_geom, which also carries them through the first half map).
// The kick-point positions are rebuilt from the stored step-start state with the same
// expressions as the forward kernels (the slice's first half map).
#include "device_common.hpp"
#include "internal.hpp"

namespace pic {

namespace {

constexpr int kBlk = 256;

// stencil weights and their derivatives d w / d u along one axis
template <int S>
__device__ __forceinline__ int stencil_d(double u, int n, double* w, double* dw) {
  const int b = stencil<S>(u, n, w);
  if constexpr (S == 1) {
    dw[0] = -1.0;
    dw[1] = 1.0;
  } else {
    const double d = u - floor(u + 0.5);
    dw[0] = -(0.5 - d);
    dw[1] = -2.0 * d;
    dw[2] = 0.5 + d;
  }
  return b;
}

// kick-point position of a step-start state: the slice's first half map (positions kept)
__device__ __forceinline__ void kick_point(const double* __restrict__ X, int64_t n, int64_t i,
                                          const HalfMap& first, double inv_g2, double r[3]) {
  double v[6];
  for (int q = 0; q < 6; ++q) v[q] = X[q * n + i];
  apply_half(first, v, inv_g2);
  r[0] = v[0];
  r[1] = v[2];
  r[2] = v[4];
}

// lam . (D x) summed over the (x, px) and (y, py) planes, D row-major per plane
__device__ __forceinline__ double plane_form(const double lm[4], const double* Dx,
                                             const double* Dy, const double v[4]) {
  return lm[0] * (Dx[0] * v[0] + Dx[1] * v[1]) + lm[1] * (Dx[2] * v[0] + Dx[3] * v[1]) +
         lm[2] * (Dy[0] * v[2] + Dy[1] * v[3]) + lm[3] * (Dy[2] * v[2] + Dy[3] * v[3]);
}

// one partial per block of a per-thread sum (blockDim.x == kBlk)
__device__ __forceinline__ void block_partial(double acc, double* __restrict__ partial) {
  __shared__ double sh[kBlk / 64];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int q = 0; q < kBlk / 64; ++q) s += sh[q];
    partial[blockIdx.x] = s;
  }
}

// Running extremes of the kick-point positions with the first index attaining each:
// slots 0..2 the min of x, y, z, slots 3..5 the max.
struct Extremes {
  double v[6];
  int64_t i[6];
};

__device__ __forceinline__ void ext_init(Extremes& ex) {
  for (int a = 0; a < 3; ++a) {
    ex.v[a] = INFINITY;
    ex.v[3 + a] = -INFINITY;
    ex.i[a] = ex.i[3 + a] = INT64_MAX;
  }
}

// slot q of (v, i) merged into ex: the smaller value (min slots) or the larger (max slots),
// the smaller index on a tie
__device__ __forceinline__ void ext_merge(Extremes& ex, int q, double v, int64_t i) {
  const bool better = q < 3 ? v < ex.v[q] : v > ex.v[q];
  if (better || (v == ex.v[q] && i < ex.i[q])) {
    ex.v[q] = v;
    ex.i[q] = i;
  }
}

// one slot as a (value, index) pair: min slots (q < 3) keep the smaller value, max slots the
// larger, the smaller index on a tie (the merge of ext_merge for a slot chosen at run time,
// without an array indexed by it)
__device__ __forceinline__ void ext_merge1(bool is_min, double& bv, int64_t& bi, double v,
                                           int64_t i) {
  const bool better = is_min ? v < bv : v > bv;
  if (better || (v == bv && i < bi)) {
    bv = v;
    bi = i;
  }
}

__device__ __forceinline__ void ext_update(Extremes& ex, const double r[3], int64_t i) {
  for (int a = 0; a < 3; ++a) {
    ext_merge(ex, a, r[a], i);
    ext_merge(ex, 3 + a, r[a], i);
  }
}

// block-wide merge; partial[blk 12 + q] = value, partial[blk 12 + 6 + q] = index (exact as a
// double below 2^53)
__device__ __forceinline__ void ext_block_partial(Extremes& ex, double* __restrict__ partial) {
  __shared__ double sv[kBlk / 64][6];
  __shared__ int64_t si[kBlk / 64][6];
  for (int q = 0; q < 6; ++q)
    for (int off = 32; off > 0; off >>= 1) {
      const double v = __shfl_xor(ex.v[q], off);
      const int64_t i = __shfl_xor(ex.i[q], off);
      ext_merge(ex, q, v, i);
    }
  if ((threadIdx.x & 63) == 0)
    for (int q = 0; q < 6; ++q) {
      sv[threadIdx.x >> 6][q] = ex.v[q];
      si[threadIdx.x >> 6][q] = ex.i[q];
    }
  __syncthreads();
  if (threadIdx.x < 6) {
    const int q = threadIdx.x;
    double bv = q < 3 ? INFINITY : -INFINITY;
    int64_t bi = INT64_MAX;
    for (int w = 0; w < kBlk / 64; ++w) ext_merge1(q < 3, bv, bi, sv[w][q], si[w][q]);
    partial[blockIdx.x * 12 + q] = bv;
    partial[blockIdx.x * 12 + 6 + q] = (double)bi;
  }
}

// out[q] = the index of extreme q = blockIdx.x over the block partials: one wave per slot, lane
// l merging blocks l, l + 64, ..., then a butterfly; the merge (better value, lower index on a
// tie) is a total order, so the result does not depend on the order of the merges
__global__ void k_ext_combine(const double* __restrict__ partial, int nblocks,
                              double* __restrict__ out) {
  const int q = blockIdx.x;
  double bv = q < 3 ? INFINITY : -INFINITY;
  int64_t bi = INT64_MAX;
  for (int b = threadIdx.x; b < nblocks; b += 64)
    ext_merge1(q < 3, bv, bi, partial[b * 12 + q], (int64_t)partial[b * 12 + 6 + q]);
  for (int off = 32; off > 0; off >>= 1) {
    const double v = __shfl_xor(bv, off);
    const int64_t i = __shfl_xor(bi, off);
    ext_merge1(q < 3, bv, bi, v, i);
  }
  if (threadIdx.x == 0) out[q] = (double)bi;
}

// out[q] = sum over b < nblocks of partial[b sb + q sq] for column q = blockIdx.x: one wave per
// column, lane l summing b = l, l + 64, ..., then a fixed butterfly (the order does not depend
// on timing)
__global__ void k_combine_cols(const double* __restrict__ partial, int nblocks, int64_t sb,
                               int64_t sq, double* __restrict__ out) {
  const int q = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += 64) s += partial[b * sb + q * sq];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if (threadIdx.x == 0) out[q] = s;
}

// block partials of ncomp grid dot products: partial[blk ncomp + c] = sum_i a[c stride + i]
// b[c stride + i] over this block's share of i < count
template <typename T>
__global__ __launch_bounds__(kBlk) void k_grid_dot(const T* __restrict__ a,
                                                   const T* __restrict__ b, int64_t count,
                                                   int ncomp, int64_t stride,
                                                   double* __restrict__ partial) {
  __shared__ double sh[kBlk / 64];
  for (int c = 0; c < ncomp; ++c) {
    double acc = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kBlk + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * kBlk)
      acc += (double)a[c * stride + i] * (double)b[c * stride + i];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int w = 0; w < kBlk / 64; ++w) t += sh[w];
      partial[blockIdx.x * ncomp + c] = t;
    }
  }
}

// The second half map's strength term of a quadrupole slice: sum_i lam_i . DG x_next,i with
// DG = (d second/dk) second^-1 and x_next the state after the slice.
__global__ __launch_bounds__(kBlk) void k_adj_dk_second(const double* __restrict__ Xn,
                                                        const double* __restrict__ lam, Consts c,
                                                        AdjSlice sl,
                                                        double* __restrict__ dk_partial) {
  const int64_t n = c.n;
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kBlk + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlk) {
    const double lm[4] = {lam[i], lam[n + i], lam[2 * n + i], lam[3 * n + i]};
    const double v[4] = {Xn[i], Xn[n + i], Xn[2 * n + i], Xn[3 * n + i]};
    acc += plane_form(lm, sl.dgx, sl.dgy, v);
  }
  block_partial(acc, dk_partial);
}

template <typename T>
__device__ __forceinline__ void add_global(T* p, T v) {
  unsafeAtomicAdd(p, v);
}

// Pass A: lam <- drift_T(lam, L/2); e += W a at the kick point.
template <int S, typename T>
__global__ __launch_bounds__(kBlk) void k_adj_a(const double* __restrict__ X,
                                                double* __restrict__ lam,
                                                const Geom* __restrict__ g, Consts c,
                                                AdjSlice sl, T* __restrict__ e,
                                                double* __restrict__ ext_partial) {
  if (g->status) return;
  const double o[3] = {g->origin[0], g->origin[1], g->origin[2]};
  const double ih[3] = {g->inv_h[0], g->inv_h[1], g->inv_h[2]};
  const int64_t n = c.n;
  const int64_t ng = (int64_t)c.nx * c.ny * c.nz;
  const double L = sl.L;
  Extremes ex;
  ext_init(ex);
  for (int64_t i = blockIdx.x * (int64_t)kBlk + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlk) {
    double r[3];
    kick_point(X, n, i, sl.first, c.inv_gamma2, r);
    ext_update(ex, r, i);
    double lm[6];
    for (int q = 0; q < 6; ++q) lm[q] = lam[q * n + i];
    apply_half_T(sl.second, lm, c.inv_gamma2);
    for (int q = 0; q < 6; ++q) lam[q * n + i] = lm[q];
    const double a[3] = {c.C * L * lm[1], c.C * L * lm[3], c.gamma * c.C * L * lm[5]};
    double wx[S + 1], wy[S + 1], wz[S + 1];
    const int bx = stencil<S>((r[0] - o[0]) * ih[0], c.nx, wx);
    const int by = stencil<S>((r[1] - o[1]) * ih[1], c.ny, wy);
    const int bz = stencil<S>((r[2] - o[2]) * ih[2], c.nz, wz);
    for (int za = 0; za <= S; ++za)
      for (int yb = 0; yb <= S; ++yb) {
        const double wzy = wz[za] * wy[yb];
        const int64_t row = ((int64_t)(bz + za) * c.ny + (by + yb)) * c.nx + bx;
        for (int q = 0; q <= S; ++q) {
          const double w = wzy * wx[q];
          add_global(&e[row + q], (T)(w * a[0]));
          add_global(&e[ng + row + q], (T)(w * a[1]));
          add_global(&e[2 * ng + row + q], (T)(w * a[2]));
        }
      }
  }
  ext_block_partial(ex, ext_partial);
}

// Pass A for the binned vector deposit: lam <- (second half map)^T lam, and the particle's
// kick-point position and a = (C L lam_px, C L lam_py, gamma C L lam_delta) written as the rows
// (r_x, a_x, r_y, a_y, r_z, a_z) of P, the layout the binning and the tiled deposit read.
__global__ __launch_bounds__(kBlk) void k_adj_stage(const double* __restrict__ X,
                                                    double* __restrict__ lam,
                                                    const Geom* __restrict__ g, Consts c,
                                                    AdjSlice sl, double* __restrict__ P,
                                                    double* __restrict__ ext_partial) {
  if (g->status) return;
  const int64_t n = c.n;
  const double L = sl.L;
  Extremes ex;
  ext_init(ex);
  for (int64_t i = blockIdx.x * (int64_t)kBlk + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlk) {
    double r[3];
    kick_point(X, n, i, sl.first, c.inv_gamma2, r);
    ext_update(ex, r, i);
    double lm[6];
    for (int q = 0; q < 6; ++q) lm[q] = lam[q * n + i];
    apply_half_T(sl.second, lm, c.inv_gamma2);
    for (int q = 0; q < 6; ++q) lam[q * n + i] = lm[q];
    P[i] = r[0];
    P[n + i] = c.C * L * lm[1];
    P[2 * n + i] = r[1];
    P[3 * n + i] = c.C * L * lm[3];
    P[4 * n + i] = r[2];
    P[5 * n + i] = c.gamma * c.C * L * lm[5];
  }
  ext_block_partial(ex, ext_partial);
}

// psi on nodes -1..n ([(nz+2)][(ny+2)][(nx+2)]) = sum_c (e_c(m + 1_c) - e_c(m - 1_c)) / (2 h_c),
// e_c = 0 outside nodes 0..n-1 (rest-frame spacings).
template <typename T>
__global__ __launch_bounds__(kBlk) void k_adj_div(const Geom* __restrict__ g,
                                                  const T* __restrict__ e, T* __restrict__ psi,
                                                  int nx, int ny, int nz) {
  if (g->status) return;
  const int px = nx + 2, py = ny + 2, pz = nz + 2;
  const int64_t total = (int64_t)px * py * pz;
  const int64_t ng = (int64_t)nx * ny * nz;
  const double cx = 1.0 / (2.0 * g->h_rest[0]);
  const double cy = 1.0 / (2.0 * g->h_rest[1]);
  const double cz = 1.0 / (2.0 * g->h_rest[2]);
  for (int64_t t = blockIdx.x * (int64_t)kBlk + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * kBlk) {
    const int i = (int)(t % px) - 1, j = (int)((t / px) % py) - 1, k = (int)(t / ((int64_t)px * py)) - 1;
    auto at = [&](int comp, int ii, int jj, int kk) -> double {
      if (ii < 0 || ii >= nx || jj < 0 || jj >= ny || kk < 0 || kk >= nz) return 0.0;
      return (double)e[comp * ng + ((int64_t)kk * ny + jj) * nx + ii];
    };
    const double v = (at(0, i + 1, j, k) - at(0, i - 1, j, k)) * cx +
                     (at(1, i, j + 1, k) - at(1, i, j - 1, k)) * cy +
                     (at(2, i, j, k + 1) - at(2, i, j, k - 1)) * cz;
    psi[t] = (T)v;
  }
}

// Pass B: lam_r += sum grad W (a . E') + q sum grad W chi at the kick point; then the first
// half map's strength term (thin: sum(-x lam_px + y lam_py) between the transposed drift and
// the transposed thin quad; quadrupole: sum lam . (d first/dk) x at the step start) into the
// block's dk partial, and lam <- (first half map)^T lam.
template <int S, typename T>
__global__ __launch_bounds__(kBlk) void k_adj_b(const double* __restrict__ X,
                                                double* __restrict__ lam,
                                                const Geom* __restrict__ g, Consts c,
                                                AdjSlice sl, const T* __restrict__ E,
                                                const T* __restrict__ chi,
                                                double* __restrict__ dk_partial,
                                                double* __restrict__ geo_partial) {
  double acc = 0.0;
  double sg[3] = {0.0, 0.0, 0.0}, sgu[3] = {0.0, 0.0, 0.0};  // sum g_a, sum g_a u_a
  if (g->status == 0) {
    const double o[3] = {g->origin[0], g->origin[1], g->origin[2]};
    const double ih[3] = {g->inv_h[0], g->inv_h[1], g->inv_h[2]};
    const int64_t n = c.n;
    const int64_t ng = (int64_t)c.nx * c.ny * c.nz;
    const double L = sl.L;
    for (int64_t i = blockIdx.x * (int64_t)kBlk + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlk) {
      double r[3];
      kick_point(X, n, i, sl.first, c.inv_gamma2, r);
      double lm[6];
      for (int q = 0; q < 6; ++q) lm[q] = lam[q * n + i];
      const double a[3] = {c.C * L * lm[1], c.C * L * lm[3], c.gamma * c.C * L * lm[5]};
      double wx[S + 1], wy[S + 1], wz[S + 1], dx[S + 1], dy[S + 1], dz[S + 1];
      const int bx = stencil_d<S>((r[0] - o[0]) * ih[0], c.nx, wx, dx);
      const int by = stencil_d<S>((r[1] - o[1]) * ih[1], c.ny, wy, dy);
      const int bz = stencil_d<S>((r[2] - o[2]) * ih[2], c.nz, wz, dz);
      double gx = 0.0, gy = 0.0, gz = 0.0;
      for (int za = 0; za <= S; ++za)
        for (int yb = 0; yb <= S; ++yb) {
          const int64_t row = ((int64_t)(bz + za) * c.ny + (by + yb)) * c.nx + bx;
          for (int q = 0; q <= S; ++q) {
            const int64_t node = row + q;
            const double s = a[0] * (double)E[node] + a[1] * (double)E[ng + node] +
                             a[2] * (double)E[2 * ng + node] + c.q_macro * (double)chi[node];
            gx += (dx[q] * ih[0]) * wy[yb] * wz[za] * s;
            gy += wx[q] * (dy[yb] * ih[1]) * wz[za] * s;
            gz += wx[q] * wy[yb] * (dz[za] * ih[2]) * s;
          }
        }
      lm[0] += gx;
      lm[2] += gy;
      lm[4] += gz;
      const double gv[3] = {gx, gy, gz};
      for (int q = 0; q < 3; ++q) {
        sg[q] += gv[q];
        sgu[q] += gv[q] * ((r[q] - o[q]) * ih[q]);
      }
      if (sl.first.type == kHalfThinDrift) {
        // transposed first half drift, the strength term with the step-start positions, then
        // the transposed thin quad
        const double ell = sl.first.ell;
        lm[1] += ell * lm[0];
        lm[3] += ell * lm[2];
        lm[5] += ell * lm[4] * c.inv_gamma2;
        const double x = X[i], y = X[2 * n + i];
        acc += -x * lm[1] + y * lm[3];
        lm[0] -= sl.first.k * lm[1];
        lm[2] += sl.first.k * lm[3];
      } else {
        if (sl.dk_kind == kDkMatrix) {
          const double v[4] = {X[i], X[n + i], X[2 * n + i], X[3 * n + i]};
          acc += plane_form(lm, sl.dfx, sl.dfy, v);
        }
        apply_half_T(sl.first, lm, c.inv_gamma2);
      }
      for (int q = 0; q < 6; ++q) lam[q * n + i] = lm[q];
    }
  }
  block_partial(acc, dk_partial);
  for (int q = 0; q < 6; ++q) {
    __syncthreads();
    block_partial(q < 3 ? sg[q] : sgu[q - 3], geo_partial + q * gridDim.x);
  }
}

// The geometry's terms of one reverse step, one thread.  geo: [0..5] indices of the particles
// at the box's min (x, y, z) and max, [6..8] sum g_a, [9..11] sum g_a u_a, [12..14] dJ/dh'_b
// through the kernel, [15..17] sum_n e_b E'_b (the centred difference's term is minus that over
// h'_b; zero for the direct field).  dJ/dmin and dJ/dmax are added to
// those particles' kick-point position adjoints, carried through the slice's first half map
// as k_adj_b carries every particle's (lam already holds the step-start adjoint), with the
// first half map's strength term into dk[sl.elem].
__global__ void k_adj_geom(const double* __restrict__ X, double* __restrict__ lam,
                           const Geom* __restrict__ g, Consts c, AdjSlice sl,
                           const double* __restrict__ geo, double* __restrict__ dk) {
  if (blockIdx.x != 0 || threadIdx.x != 0 || g->status) return;
  const int64_t n = c.n;
  const double nodes[3] = {(double)c.nx, (double)c.ny, (double)c.nz};
  const double dhr[3] = {1.0, 1.0, c.gamma};  // d h'_a / d h_a
  double dmin[3], dmax[3];
  for (int a = 0; a < 3; ++a) {
    const double dJ_do = -geo[6 + a];
    const double dJ_dhr = geo[12 + a] - geo[15 + a] / g->h_rest[a];
    const double dJ_dh = -geo[9 + a] + dJ_dhr * dhr[a];
    const double m = nodes[a] - 3.5;
    dmin[a] = dJ_do * (1.0 + 1.25 / m) - dJ_dh / m;
    dmax[a] = -dJ_do * 1.25 / m + dJ_dh / m;
  }
  double acc = 0.0;
  for (int q = 0; q < 6; ++q) {
    const int a = q % 3;
    const int64_t i = (int64_t)geo[q];
    if (i < 0 || i >= n) continue;  // no particle (cannot happen for n >= 1)
    double d[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    d[2 * a] = q < 3 ? dmin[a] : dmax[a];
    if (sl.first.type == kHalfThinDrift) {
      const double ell = sl.first.ell;
      d[1] += ell * d[0];
      d[3] += ell * d[2];
      d[5] += ell * d[4] * c.inv_gamma2;
      acc += -X[i] * d[1] + X[2 * n + i] * d[3];
      d[0] -= sl.first.k * d[1];
      d[2] += sl.first.k * d[3];
    } else {
      if (sl.dk_kind == kDkMatrix) {
        const double v[4] = {X[i], X[n + i], X[2 * n + i], X[3 * n + i]};
        acc += plane_form(d, sl.dfx, sl.dfy, v);
      }
      apply_half_T(sl.first, d, c.inv_gamma2);
    }
    for (int r = 0; r < 6; ++r) lam[r * n + i] += d[r];
  }
  if (sl.dk_kind != kDkNone) dk[sl.elem] += acc;
}

// dk[slot] += sum of the per-block partials: one wave, lane l sums partials l, l + 64, ...,
// then a fixed butterfly (the summation order does not depend on timing)
__global__ void k_adj_dk_combine(const double* __restrict__ partial, int nblocks,
                                 double* __restrict__ dk, int slot) {
  double s = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += 64) s += partial[b];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if (threadIdx.x == 0) dk[slot] += s;
}

// lam = dJ/dX of J = w . (sigma_x, sigma_y, eps_x, eps_y); mom = [mean 6][cov upper 21]
struct Weights {
  double w[4];
};

// covariance entry (a, b) of mom = [mean 6][cov upper 21] (upper triangle, row-major, a <= b)
__device__ __forceinline__ double mom_cov(const double* __restrict__ mom, int a, int b) {
  if (a > b) {
    int t = a;
    a = b;
    b = t;
  }
  int q = 0;
  for (int r = 0; r < a; ++r) q += 6 - r;
  return mom[6 + q + (b - a)];
}

// The objective terms of the final beam: centred rms sizes and geometric (unnormalised)
// emittances, eps_x = sqrt(<dx^2><dpx^2> - <dx dpx>^2) (the paper quotes the emittance in this
// unnormalised form: sections "Usage Example" and "Benchmark: FODO Cell").  One thread.
__global__ void k_objective(const double* __restrict__ mom, double* __restrict__ out_m) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  const double Sxx = mom_cov(mom, 0, 0), Sxp = mom_cov(mom, 0, 1), Spp = mom_cov(mom, 1, 1);
  const double Syy = mom_cov(mom, 2, 2), Syq = mom_cov(mom, 2, 3), Sqq = mom_cov(mom, 3, 3);
  out_m[0] = sqrt(Sxx);
  out_m[1] = sqrt(Syy);
  out_m[2] = sqrt(Sxx * Spp - Sxp * Sxp);
  out_m[3] = sqrt(Syy * Sqq - Syq * Syq);
}

__global__ __launch_bounds__(kBlk) void k_obj_grad(const double* __restrict__ X, int64_t n,
                                                   const double* __restrict__ mom, Weights wt,
                                                   double* __restrict__ lam,
                                                   double* __restrict__ out_m) {
  auto cov = [&](int a, int b) { return mom_cov(mom, a, b); };
  const double Sxx = cov(0, 0), Sxp = cov(0, 1), Spp = cov(1, 1);
  const double Syy = cov(2, 2), Syq = cov(2, 3), Sqq = cov(3, 3);
  const double sx = sqrt(Sxx), sy = sqrt(Syy);
  const double ex = sqrt(Sxx * Spp - Sxp * Sxp), ey = sqrt(Syy * Sqq - Syq * Syq);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    out_m[0] = sx;
    out_m[1] = sy;
    out_m[2] = ex;
    out_m[3] = ey;
  }
  const double inv_n = 1.0 / (double)n;
  for (int64_t i = blockIdx.x * (int64_t)kBlk + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlk) {
    const double dxv = X[i] - mom[0], dpx = X[n + i] - mom[1];
    const double dyv = X[2 * n + i] - mom[2], dpy = X[3 * n + i] - mom[3];
    lam[i] = wt.w[0] * dxv * inv_n / sx + wt.w[2] * (Spp * dxv - Sxp * dpx) * inv_n / ex;
    lam[n + i] = wt.w[2] * (Sxx * dpx - Sxp * dxv) * inv_n / ex;
    lam[2 * n + i] = wt.w[1] * dyv * inv_n / sy + wt.w[3] * (Sqq * dyv - Syq * dpy) * inv_n / ey;
    lam[3 * n + i] = wt.w[3] * (Syy * dpy - Syq * dyv) * inv_n / ey;
    lam[4 * n + i] = 0.0;
    lam[5 * n + i] = 0.0;
  }
}

// partial[b][36] = per-block sums of lam_a xi_b (dJ/dL = lam0 xi^T)
__global__ __launch_bounds__(kBlk) void k_dL(const double* __restrict__ lam,
                                             const double* __restrict__ xi, int64_t n,
                                             double* __restrict__ partial) {
  __shared__ double sh[kBlk / 64];
  double s[36];
  for (int q = 0; q < 36; ++q) s[q] = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kBlk + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlk) {
    double l[6], x[6];
    for (int r = 0; r < 6; ++r) {
      l[r] = lam[r * n + i];
      x[r] = xi[r * n + i];
    }
    for (int a = 0; a < 6; ++a)
      for (int b = 0; b < 6; ++b) s[a * 6 + b] += l[a] * x[b];
  }
#pragma unroll
  for (int q = 0; q < 36; ++q) {
    double v = s[q];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int w = 0; w < kBlk / 64; ++w) t += sh[w];
      partial[blockIdx.x * 36 + q] = t;
    }
  }
}

__global__ void k_dL_combine(const double* __restrict__ partial, int nblocks,
                             double* __restrict__ out) {
  const int q = threadIdx.x;
  if (q >= 36) return;
  double s = 0.0;
  for (int b = 0; b < nblocks; ++b) s += partial[b * 36 + q];
  out[q] = s;
}

int grid_for(int64_t n) {
  int64_t b = (n + kBlk - 1) / kBlk;
  if (b > kAdjBlocks) b = kAdjBlocks;
  return (int)(b < 1 ? 1 : b);
}

}  // namespace

hipError_t launch_adj_dk_second(const double* Xnext, const double* lam, Consts c,
                                const AdjSlice& sl, double* dk_partial, double* dk,
                                hipStream_t s) {
  if (sl.dk_kind != kDkMatrix) return hipSuccess;
  const int nb = grid_for(c.n);
  hipLaunchKernelGGL(k_adj_dk_second, dim3(nb), dim3(kBlk), 0, s, Xnext, lam, c, sl, dk_partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_adj_dk_combine, dim3(1), dim3(64), 0, s, dk_partial, nb, dk, sl.elem);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_adj_a(const double* X, double* lam, const Geom* g, Consts c,
                        const AdjSlice& sl, T* e, double* ext_partial, double* geo,
                        hipStream_t s) {
  const int nb = grid_for(c.n);
  if (c.shape == 1)
    hipLaunchKernelGGL((k_adj_a<1, T>), dim3(nb), dim3(kBlk), 0, s, X, lam, g, c, sl, e,
                       ext_partial);
  else
    hipLaunchKernelGGL((k_adj_a<2, T>), dim3(nb), dim3(kBlk), 0, s, X, lam, g, c, sl, e,
                       ext_partial);
  PIC_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_ext_combine, dim3(6), dim3(64), 0, s, ext_partial, nb, geo);
  return hipGetLastError();
}

hipError_t launch_adj_stage(const double* X, double* lam, const Geom* g, Consts c,
                            const AdjSlice& sl, double* P, double* ext_partial, double* geo,
                            hipStream_t s) {
  const int nb = grid_for(c.n);
  hipLaunchKernelGGL(k_adj_stage, dim3(nb), dim3(kBlk), 0, s, X, lam, g, c, sl, P, ext_partial);
  PIC_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_ext_combine, dim3(6), dim3(64), 0, s, ext_partial, nb, geo);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_grid_dot(const T* a, const T* b, int64_t count, int ncomp, int64_t stride,
                           double* partial, double* out, hipStream_t s) {
  const int nb = grid_for(count);
  hipLaunchKernelGGL((k_grid_dot<T>), dim3(nb), dim3(kBlk), 0, s, a, b, count, ncomp, stride,
                     partial);
  PIC_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_combine_cols, dim3(ncomp), dim3(64), 0, s, partial, nb, (int64_t)ncomp,
                     (int64_t)1, out);
  return hipGetLastError();
}

hipError_t launch_adj_geom(const double* X, double* lam, const Geom* g, Consts c,
                           const AdjSlice& sl, const double* geo, double* dk, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_geom, dim3(1), dim3(64), 0, s, X, lam, g, c, sl, geo, dk);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_adj_div(const Geom* g, const T* e, T* psi, int nx, int ny, int nz,
                          hipStream_t s) {
  const int64_t total = (int64_t)(nx + 2) * (ny + 2) * (nz + 2);
  hipLaunchKernelGGL((k_adj_div<T>), dim3(grid_for(total)), dim3(kBlk), 0, s, g, e, psi, nx, ny,
                     nz);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_adj_b(const double* X, double* lam, const Geom* g, Consts c, const AdjSlice& sl,
                        const T* E, const T* chi, double* dk_partial, double* dk,
                        double* geo_partial, double* geo, hipStream_t s) {
  const int nb = grid_for(c.n);
  if (c.shape == 1)
    hipLaunchKernelGGL((k_adj_b<1, T>), dim3(nb), dim3(kBlk), 0, s, X, lam, g, c, sl, E, chi,
                       dk_partial, geo_partial);
  else
    hipLaunchKernelGGL((k_adj_b<2, T>), dim3(nb), dim3(kBlk), 0, s, X, lam, g, c, sl, E, chi,
                       dk_partial, geo_partial);
  PIC_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_adj_dk_combine, dim3(1), dim3(64), 0, s, dk_partial, nb, dk, sl.elem);
  PIC_TRY(hipGetLastError());
  // geo_partial[q nb + b] (q = 0..5) summed over the blocks into geo[6 + q]
  hipLaunchKernelGGL(k_combine_cols, dim3(6), dim3(64), 0, s, geo_partial, nb, (int64_t)1,
                     (int64_t)nb, geo + 6);
  return hipGetLastError();
}

hipError_t launch_obj_grad(const double* X, int64_t n, const double* mom, const double w[4],
                           double* lam, double* out_m, hipStream_t s) {
  Weights wt;
  for (int q = 0; q < 4; ++q) wt.w[q] = w[q];
  hipLaunchKernelGGL(k_obj_grad, dim3(grid_for(n)), dim3(kBlk), 0, s, X, n, mom, wt, lam, out_m);
  return hipGetLastError();
}

hipError_t launch_objective(const double* mom, double* out_m, hipStream_t s) {
  hipLaunchKernelGGL(k_objective, dim3(1), dim3(64), 0, s, mom, out_m);
  return hipGetLastError();
}

hipError_t launch_dL(const double* lam, const double* xi, int64_t n, double* partial, double* out,
                     hipStream_t s) {
  const int nb = grid_for(n);
  hipLaunchKernelGGL(k_dL, dim3(nb), dim3(kBlk), 0, s, lam, xi, n, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_dL_combine, dim3(1), dim3(64), 0, s, partial, nb, out);
  return hipGetLastError();
}

template hipError_t launch_adj_a<double>(const double*, double*, const Geom*, Consts,
                                         const AdjSlice&, double*, double*, double*, hipStream_t);
template hipError_t launch_adj_a<float>(const double*, double*, const Geom*, Consts,
                                        const AdjSlice&, float*, double*, double*, hipStream_t);
template hipError_t launch_grid_dot<double>(const double*, const double*, int64_t, int, int64_t,
                                            double*, double*, hipStream_t);
template hipError_t launch_grid_dot<float>(const float*, const float*, int64_t, int, int64_t,
                                           double*, double*, hipStream_t);
template hipError_t launch_adj_div<double>(const Geom*, const double*, double*, int, int, int,
                                           hipStream_t);
template hipError_t launch_adj_div<float>(const Geom*, const float*, float*, int, int, int,
                                          hipStream_t);
template hipError_t launch_adj_b<double>(const double*, double*, const Geom*, Consts,
                                         const AdjSlice&, const double*, const double*, double*,
                                         double*, double*, double*, hipStream_t);
template hipError_t launch_adj_b<float>(const double*, double*, const Geom*, Consts,
                                        const AdjSlice&, const float*, const float*, double*,
                                        double*, double*, double*, hipStream_t);

}  // namespace pic
