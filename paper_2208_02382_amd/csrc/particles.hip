// Particle kernels: beam initialisation, box reduction and geometry, field gather, linear
// maps (drift, thin quadrupole, space-charge kick) and beam moments.  (The charge deposition
// is binned by tile, in sort.hip.)
//
// Phase space is structure-of-arrays float64 X[6][n] = (x, px, y, py, z, delta); every kernel
// walks particles with a grid-stride loop so consecutive lanes touch consecutive doubles of
// each row (coalesced 64-lane reads of 512 B per row).
#include "device_common.hpp"
#include "internal.hpp"

namespace pic {

namespace {

constexpr int kBlock = 256;

int grid_for(int64_t n) {
  int64_t b = (n + kBlock - 1) / kBlock;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return (int)b;
}

// ---------------------------------------------------------------------------- box and geometry

__global__ void k_box_reset(Box* box) {
  int t = threadIdx.x;
  if (t < 3) {
    box->mn[t] = ~0ull;
    box->mx[t] = 0ull;
  }
  if (t == 0) box->nonfinite = 0u;
}

__global__ __launch_bounds__(kBlock) void k_box(const double* __restrict__ X, int64_t n, Box* box) {
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  bool bad = false;
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock) {
    double p[3] = {X[i], X[2 * n + i], X[4 * n + i]};
    for (int a = 0; a < 3; ++a) {
      bad |= !isfinite(p[a]);
      lo[a] = fmin(lo[a], p[a]);
      hi[a] = fmax(hi[a], p[a]);
    }
  }
  box_accumulate_block(lo, hi, bad, box);
}

// Geometry from the box: h = (max - min)/(n - 3.5), node 0 at min - 1.25 h (the extreme
// particles sit a quarter cell from a node and from a cell boundary: inside every stencil, on
// no kink of the CIC or TSC weights); the rest-frame cell is (hx, hy, gamma hz).  A non-finite coordinate or a zero extent sets status = -4 (PIC_EDOMAIN),
// which is sticky until the beam is initialised again.
// The origin's product and difference are rounded separately (no fused multiply-add), as a
// plain float64 evaluation of the same formula does.
__device__ void geometry_from_box(const Box* box, Geom* g, const Consts& c) {
#pragma clang fp contract(off)
  int nn[3] = {c.nx, c.ny, c.nz};
  bool bad = box->nonfinite != 0u;
  double lo[3], hi[3];
  for (int a = 0; a < 3; ++a) {
    lo[a] = ord_dec(box->mn[a]);
    hi[a] = ord_dec(box->mx[a]);
    if (!(hi[a] > lo[a])) bad = true;
  }
  if (bad) {
    g->status = -4;
    return;
  }
  for (int a = 0; a < 3; ++a) {
    const double h = (hi[a] - lo[a]) / ((double)nn[a] - 3.5);
    g->h[a] = h;
    g->inv_h[a] = 1.0 / h;
    g->origin[a] = lo[a] - 1.25 * h;
  }
  g->h_rest[0] = g->h[0];
  g->h_rest[1] = g->h[1];
  g->h_rest[2] = c.gamma * g->h[2];
}

__global__ void k_geometry(const Box* box, Geom* g, Consts c) {
  if (threadIdx.x != 0) return;
  geometry_from_box(box, g, c);
}

// ---------------------------------------------------------------------------- initialisation

__global__ void k_clear_status(Geom* g) {
  if (threadIdx.x == 0) g->status = 0;
}

__global__ __launch_bounds__(kBlock) void k_init_normals(double* __restrict__ X,
                                                         const double* __restrict__ xi, int64_t n,
                                                         Chol L) {
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock) {
    double v[6];
    for (int r = 0; r < 6; ++r) v[r] = xi[r * n + i];
    for (int r = 0; r < 6; ++r) {
      double s = 0.0;
      for (int q = 0; q <= r; ++q) s += L.L[r * 6 + q] * v[q];
      X[r * n + i] = s;
    }
  }
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of the 4x32 S-box with
// multipliers 0xD2511F53, 0xCD9E8D57 and key increments 0x9E3779B9, 0xBB67AE85.
__device__ __forceinline__ void philox4x32_10(unsigned c[4], unsigned k0, unsigned k1) {
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    unsigned lo0 = 0xD2511F53u * c[0], hi0 = __umulhi(0xD2511F53u, c[0]);
    unsigned lo1 = 0xCD9E8D57u * c[2], hi1 = __umulhi(0xCD9E8D57u, c[2]);
    unsigned n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

// 53-bit uniform in (0, 1] from two words: ((a >> 5) 2^26 + (b >> 6) + 1) 2^-53.
__device__ __forceinline__ double u53(unsigned a, unsigned b) {
  unsigned long long k = ((unsigned long long)(a >> 5) << 26) + (unsigned long long)(b >> 6) + 1ull;
  return (double)k * 0x1.0p-53;
}

// dist 0: Gaussian core (Box-Muller of draw blocks 0-2) and, for i >= n_core, the uniform
// halo in [-4, 4]^6.  dist 1: Waterbag, uniform in the 6-ball of radius sqrt(8) (unit
// covariance): the direction of the six normals times sqrt(8) u^(1/6), u from draw block 3.
__global__ __launch_bounds__(kBlock) void k_init_philox(double* __restrict__ X, int64_t n,
                                                        int64_t n_core, unsigned k0, unsigned k1,
                                                        Chol L, int dist) {
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock) {
    double v[6];
    bool core = dist == 1 || i < n_core;
    for (unsigned blk = 0; blk < 3; ++blk) {
      unsigned c[4] = {(unsigned)((unsigned long long)i & 0xffffffffull),
                       (unsigned)((unsigned long long)i >> 32), blk, 0u};
      philox4x32_10(c, k0, k1);
      double ua = u53(c[0], c[1]);
      double ub = u53(c[2], c[3]);
      if (core) {
        double rad = sqrt(-2.0 * log(ua));
        double s, co;
        sincospi(2.0 * ub, &s, &co);
        v[2 * blk] = rad * co;
        v[2 * blk + 1] = rad * s;
      } else {
        v[2 * blk] = -4.0 + 8.0 * ua;
        v[2 * blk + 1] = -4.0 + 8.0 * ub;
      }
    }
    if (dist == 1) {
      unsigned c[4] = {(unsigned)((unsigned long long)i & 0xffffffffull),
                       (unsigned)((unsigned long long)i >> 32), 3u, 0u};
      philox4x32_10(c, k0, k1);
      double g2 = 0.0;
      for (int r = 0; r < 6; ++r) g2 += v[r] * v[r];
      const double scale = sqrt(8.0) * pow(u53(c[0], c[1]), 1.0 / 6.0) / sqrt(g2);
      for (int r = 0; r < 6; ++r) v[r] *= scale;
    }
    for (int r = 0; r < 6; ++r) {
      double s = 0.0;
      for (int q = 0; q <= r; ++q) s += L.L[r * 6 + q] * v[q];
      X[r * n + i] = s;
    }
  }
}

// ---------------------------------------------------------------------------- gather

// Field at the particles from E'[3][nz][ny][nx] with the deposit's weights.
template <int S, typename T>
__device__ __forceinline__ void gather_one(double x, double y, double z, const double* o,
                                           const double* ih, const T* __restrict__ E, Consts c,
                                           T out[3]) {
  double wx[S + 1], wy[S + 1], wz[S + 1];
  int bx = stencil<S>((x - o[0]) * ih[0], c.nx, wx);
  int by = stencil<S>((y - o[1]) * ih[1], c.ny, wy);
  int bz = stencil<S>((z - o[2]) * ih[2], c.nz, wz);
  const int64_t plane = (int64_t)c.nx * c.ny * c.nz;
  T ex = 0, ey = 0, ez = 0;
  for (int a = 0; a <= S; ++a)
    for (int b = 0; b <= S; ++b) {
      double wzy = wz[a] * wy[b];
      int64_t row = ((int64_t)(bz + a) * c.ny + (by + b)) * c.nx + bx;
      for (int q = 0; q <= S; ++q) {
        T w = (T)(wzy * wx[q]);
        ex += w * E[row + q];
        ey += w * E[plane + row + q];
        ez += w * E[2 * plane + row + q];
      }
    }
  out[0] = ex;
  out[1] = ey;
  out[2] = ez;
}

template <int S, typename T>
__global__ __launch_bounds__(kBlock) void k_gather(const double* __restrict__ X,
                                                   const Geom* __restrict__ g,
                                                   const T* __restrict__ E, T* __restrict__ Ep,
                                                   Consts c) {
  if (g->status) return;
  double o[3] = {g->origin[0], g->origin[1], g->origin[2]};
  double ih[3] = {g->inv_h[0], g->inv_h[1], g->inv_h[2]};
  const int64_t n = c.n;
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock) {
    T e[3];
    gather_one<S, T>(X[i], X[2 * n + i], X[4 * n + i], o, ih, E, c, e);
    Ep[i] = e[0];
    Ep[n + i] = e[1];
    Ep[2 * n + i] = e[2];
  }
}

// ---------------------------------------------------------------------------- linear maps

// drift: x += l px, y += l py, z += l delta / gamma^2
__device__ __forceinline__ void drift(double v[6], double ell, double inv_g2) {
  v[0] = v[0] + ell * v[1];
  v[2] = v[2] + ell * v[3];
  v[4] = v[4] + ell * v[5] * inv_g2;
}

// thin quadrupole of integrated strength k: px -= k x, py += k y
__device__ __forceinline__ void thin_quad(double v[6], double k) {
  v[1] = v[1] - k * v[0];
  v[3] = v[3] + k * v[2];
}

// space-charge kick over L: px += C E'x L, py += C E'y L, delta += gamma C E'z L
__device__ __forceinline__ void sc_kick(double v[6], double ex, double ey, double ez, double L,
                                        Consts c) {
  v[1] = v[1] + c.C * ex * L;
  v[3] = v[3] + c.C * ey * L;
  v[5] = v[5] + c.gamma * c.C * ez * L;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_push(double* __restrict__ X, int kind, double value,
                                                 const T* __restrict__ Ep, Consts c) {
  const int64_t n = c.n;
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock) {
    double v[6];
    for (int r = 0; r < 6; ++r) v[r] = X[r * n + i];
    if (kind == 0) drift(v, value, c.inv_gamma2);
    else if (kind == 1) thin_quad(v, value);
    else sc_kick(v, (double)Ep[i], (double)Ep[n + i], (double)Ep[2 * n + i], value, c);
    for (int r = 0; r < 6; ++r) X[r * n + i] = v[r];
  }
}

// Fused second half of step j and first half of step j+1: gather E' at the current positions,
// kick over L, the slice's second half map; if has_next, the next slice's first half map, and
// accumulate the box of the new positions (the next step's grid).  The two half maps act as
// their product (half_product), as in the tiled gather-kick, so both paths compute the same bits.
template <int S, typename T>
__global__ __launch_bounds__(kBlock) void k_gkd(double* __restrict__ X, const Geom* __restrict__ g,
                                                const T* __restrict__ E, double L, HalfMap second,
                                                int has_next, HalfMap first_next, Consts c,
                                                Box* box) {
  if (g->status) return;
  const HalfMap maps = half_product(second, first_next, has_next != 0);
  double o[3] = {g->origin[0], g->origin[1], g->origin[2]};
  double ih[3] = {g->inv_h[0], g->inv_h[1], g->inv_h[2]};
  const int64_t n = c.n;
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  bool bad = false;
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock) {
    double v[6];
    for (int r = 0; r < 6; ++r) v[r] = X[r * n + i];
    T e[3];
    gather_one<S, T>(v[0], v[2], v[4], o, ih, E, c, e);
    sc_kick(v, (double)e[0], (double)e[1], (double)e[2], L, c);
    apply_matrix(maps, v, c.inv_gamma2);
    if (has_next) {
      double p[3] = {v[0], v[2], v[4]};
      for (int a = 0; a < 3; ++a) {
        bad |= !isfinite(p[a]);
        lo[a] = fmin(lo[a], p[a]);
        hi[a] = fmax(hi[a], p[a]);
      }
    }
    for (int r = 0; r < 6; ++r) X[r * n + i] = v[r];
  }
  if (has_next) box_accumulate_block(lo, hi, bad, box);
}

// ---------------------------------------------------------------------------- moments

__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int q = 0; q < kBlock / 64; ++q) s += sh[q];
  return s;
}

// pass 1: per-block sums of the six coordinates
__global__ __launch_bounds__(kBlock) void k_mom_sum(const double* __restrict__ X, int64_t n,
                                                    double* partial) {
  __shared__ double sh[kBlock / 64];
  double s[6] = {0, 0, 0, 0, 0, 0};
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock)
    for (int r = 0; r < 6; ++r) s[r] += X[r * n + i];
  for (int r = 0; r < 6; ++r) {
    double t = block_sum(s[r], sh);
    if (threadIdx.x == 0) partial[blockIdx.x * kMomentSlots + r] = t;
  }
}

// combine the per-block partials of slot s0 + blockIdx.x (one wave per slot: lane l sums the
// partials of blocks l, l + 64, ..., then a fixed butterfly, so the order does not depend on
// timing); slots 0..5 become means
__global__ void k_mom_combine(const double* partial, int nblocks, int s0, int s1, int64_t n,
                              double* out) {
  const int s = s0 + blockIdx.x;
  if (s >= s1) return;
  double acc = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += 64) acc += partial[b * kMomentSlots + s];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if (threadIdx.x == 0) out[s] = acc / (double)n;
}

// pass 2: per-block sums of the 21 centred products (upper triangle, row-major)
__global__ __launch_bounds__(kBlock) void k_mom_cov(const double* __restrict__ X, int64_t n,
                                                    const double* __restrict__ mean,
                                                    double* partial) {
  __shared__ double sh[kBlock / 64];
  double m[6];
  for (int r = 0; r < 6; ++r) m[r] = mean[r];
  double s[21];
  for (int q = 0; q < 21; ++q) s[q] = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock) {
    double d[6];
    for (int r = 0; r < 6; ++r) d[r] = X[r * n + i] - m[r];
    int q = 0;
    for (int a = 0; a < 6; ++a)
      for (int b = a; b < 6; ++b) s[q++] += d[a] * d[b];
  }
  for (int q = 0; q < 21; ++q) {
    double t = block_sum(s[q], sh);
    if (threadIdx.x == 0) partial[blockIdx.x * kMomentSlots + 6 + q] = t;
  }
}

__global__ __launch_bounds__(kBlock) void k_copy_if_ok(const uint32_t* __restrict__ src,
                                                     uint32_t* __restrict__ dst, int64_t words,
                                                     const Geom* __restrict__ g) {
  if (g->status) return;
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < words;
       i += (int64_t)gridDim.x * kBlock)
    dst[i] = src[i];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_zero(T* p, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * kBlock)
    p[i] = T(0);
}

// batched: thread b handles beam b
__global__ void k_box_reset_batch(const BeamDev* __restrict__ beams, int nb) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  Box* box = beams[b].box;
  for (int a = 0; a < 3; ++a) {
    box->mn[a] = ~0ull;
    box->mx[a] = 0ull;
  }
  box->nonfinite = 0u;
}

__global__ void k_geometry_batch(const BeamDev* __restrict__ beams, int nb) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  geometry_from_box(beams[b].box, beams[b].geom, beams[b].c);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_zero_rho_batch(const BeamDev* __restrict__ beams) {
  const BeamDev& d = beams[blockIdx.y];
  T* p = (T*)d.rho;
  const int64_t count = (int64_t)d.c.nx * d.c.ny * d.c.nz;
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * kBlock)
    p[i] = T(0);
}

}  // namespace

// ---------------------------------------------------------------------------- launch wrappers

hipError_t launch_batch_box_reset(const BeamDev* beams, int nb, hipStream_t s) {
  hipLaunchKernelGGL(k_box_reset_batch, dim3((nb + 63) / 64), dim3(64), 0, s, beams, nb);
  return hipGetLastError();
}

hipError_t launch_batch_geometry(const BeamDev* beams, int nb, hipStream_t s) {
  hipLaunchKernelGGL(k_geometry_batch, dim3((nb + 63) / 64), dim3(64), 0, s, beams, nb);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_batch_zero_rho(const BeamDev* beams, int nb, const BatchDims& bd, hipStream_t s) {
  const int64_t ng = (int64_t)bd.max_nx * bd.max_ny * bd.max_nz;
  hipLaunchKernelGGL((k_zero_rho_batch<T>), dim3(grid_for(ng), nb), dim3(kBlock), 0, s, beams);
  return hipGetLastError();
}
template hipError_t launch_batch_zero_rho<double>(const BeamDev*, int, const BatchDims&, hipStream_t);
template hipError_t launch_batch_zero_rho<float>(const BeamDev*, int, const BatchDims&, hipStream_t);

hipError_t launch_box_reset(Box* box, hipStream_t s) {
  hipLaunchKernelGGL(k_box_reset, dim3(1), dim3(64), 0, s, box);
  return hipGetLastError();
}

hipError_t launch_box(const double* X, int64_t n, Box* box, hipStream_t s) {
  hipLaunchKernelGGL(k_box, dim3(grid_for(n)), dim3(kBlock), 0, s, X, n, box);
  return hipGetLastError();
}

hipError_t launch_geometry(const Box* box, Geom* g, Consts c, hipStream_t s) {
  hipLaunchKernelGGL(k_geometry, dim3(1), dim3(64), 0, s, box, g, c);
  return hipGetLastError();
}

hipError_t launch_init_normals(double* X, const double* xi, int64_t n, Chol L, hipStream_t s) {
  hipLaunchKernelGGL(k_init_normals, dim3(grid_for(n)), dim3(kBlock), 0, s, X, xi, n, L);
  return hipGetLastError();
}

hipError_t launch_init_philox(double* X, int64_t n, int64_t n_halo, uint64_t seed, Chol L,
                              int dist, hipStream_t s) {
  hipLaunchKernelGGL(k_init_philox, dim3(grid_for(n)), dim3(kBlock), 0, s, X, n, n - n_halo,
                     (unsigned)(seed & 0xffffffffull), (unsigned)(seed >> 32), L, dist);
  return hipGetLastError();
}

hipError_t launch_clear_status(Geom* g, hipStream_t s) {
  hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(64), 0, s, g);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gather(const double* X, const Geom* g, const T* E, T* Ep, Consts c,
                         hipStream_t s) {
  if (c.shape == 1)
    hipLaunchKernelGGL((k_gather<1, T>), dim3(grid_for(c.n)), dim3(kBlock), 0, s, X, g, E, Ep, c);
  else
    hipLaunchKernelGGL((k_gather<2, T>), dim3(grid_for(c.n)), dim3(kBlock), 0, s, X, g, E, Ep, c);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_push(double* X, int kind, double value, const T* Ep, Consts c, hipStream_t s) {
  hipLaunchKernelGGL((k_push<T>), dim3(grid_for(c.n)), dim3(kBlock), 0, s, X, kind, value, Ep, c);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gkd(double* X, const Geom* g, const T* E, double L, const HalfMap& second,
                      int has_next, const HalfMap& first_next, Consts c, Box* box, hipStream_t s) {
  if (c.shape == 1)
    hipLaunchKernelGGL((k_gkd<1, T>), dim3(grid_for(c.n)), dim3(kBlock), 0, s, X, g, E, L,
                       second, has_next, first_next, c, box);
  else
    hipLaunchKernelGGL((k_gkd<2, T>), dim3(grid_for(c.n)), dim3(kBlock), 0, s, X, g, E, L,
                       second, has_next, first_next, c, box);
  return hipGetLastError();
}

// both half maps of a slice, no kick
__global__ __launch_bounds__(kBlock) void k_half_maps(double* __restrict__ X, HalfMap first,
                                                      HalfMap second, Consts c) {
  const int64_t n = c.n;
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock) {
    double v[6];
    for (int r = 0; r < 6; ++r) v[r] = X[r * n + i];
    apply_half(first, v, c.inv_gamma2);
    apply_half(second, v, c.inv_gamma2);
    for (int r = 0; r < 6; ++r) X[r * n + i] = v[r];
  }
}

// One half map in place, with the box of the new positions (the first half of a step when the
// previous step's end state was needed on its own, for diagnostics).
__global__ __launch_bounds__(kBlock) void k_half_box(double* __restrict__ X, HalfMap h, Consts c,
                                                     Box* box) {
  const int64_t n = c.n;
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  bool bad = false;
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock) {
    double v[6];
    for (int r = 0; r < 6; ++r) v[r] = X[r * n + i];
    apply_half(h, v, c.inv_gamma2);
    for (int r = 0; r < 6; ++r) X[r * n + i] = v[r];
    const double p[3] = {v[0], v[2], v[4]};
    for (int a = 0; a < 3; ++a) {
      bad |= !isfinite(p[a]);
      lo[a] = fmin(lo[a], p[a]);
      hi[a] = fmax(hi[a], p[a]);
    }
  }
  if (box) box_accumulate_block(lo, hi, bad, box);
}

hipError_t launch_half_box(double* X, const HalfMap& h, Consts c, Box* box, hipStream_t s) {
  hipLaunchKernelGGL(k_half_box, dim3(grid_for(c.n)), dim3(kBlock), 0, s, X, h, c, box);
  return hipGetLastError();
}

hipError_t launch_half_maps(double* X, const HalfMap& first, const HalfMap& second, Consts c,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_half_maps, dim3(grid_for(c.n)), dim3(kBlock), 0, s, X, first, second, c);
  return hipGetLastError();
}

hipError_t launch_moments(const double* X, int64_t n, double* partial, double* out,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_mom_sum, dim3(kReduceBlocks), dim3(kBlock), 0, s, X, n, partial);
  hipLaunchKernelGGL(k_mom_combine, dim3(6), dim3(64), 0, s, partial, kReduceBlocks, 0, 6, n, out);
  hipLaunchKernelGGL(k_mom_cov, dim3(kReduceBlocks), dim3(kBlock), 0, s, X, n, out, partial);
  hipLaunchKernelGGL(k_mom_combine, dim3(21), dim3(64), 0, s, partial, kReduceBlocks, 6, 27, n,
                     out);
  return hipGetLastError();
}

hipError_t launch_copy_if_ok(const void* src, void* dst, size_t bytes, const Geom* g,
                             hipStream_t s) {
  const int64_t words = (int64_t)(bytes / 4);
  hipLaunchKernelGGL(k_copy_if_ok, dim3(grid_for(words)), dim3(kBlock), 0, s,
                     (const uint32_t*)src, (uint32_t*)dst, words, g);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_zero(T* p, int64_t count, hipStream_t s) {
  hipLaunchKernelGGL((k_zero<T>), dim3(grid_for(count)), dim3(kBlock), 0, s, p, count);
  return hipGetLastError();
}

template hipError_t launch_gather<double>(const double*, const Geom*, const double*, double*,
                                          Consts, hipStream_t);
template hipError_t launch_gather<float>(const double*, const Geom*, const float*, float*, Consts,
                                         hipStream_t);
template hipError_t launch_push<double>(double*, int, double, const double*, Consts, hipStream_t);
template hipError_t launch_push<float>(double*, int, double, const float*, Consts, hipStream_t);
template hipError_t launch_gkd<double>(double*, const Geom*, const double*, double, const HalfMap&,
                                       int, const HalfMap&, Consts, Box*, hipStream_t);
template hipError_t launch_gkd<float>(double*, const Geom*, const float*, double, const HalfMap&,
                                      int, const HalfMap&, Consts, Box*, hipStream_t);
template hipError_t launch_zero<double>(double*, int64_t, hipStream_t);
template hipError_t launch_zero<float>(float*, int64_t, hipStream_t);
template hipError_t launch_zero<uint32_t>(uint32_t*, int64_t, hipStream_t);

}  // namespace pic
