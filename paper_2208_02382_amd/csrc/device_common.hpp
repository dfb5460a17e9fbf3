// Device helpers shared by the particle kernels (particles.hip, sort.hip).
#pragma once
#include "internal.hpp"

namespace pic {

constexpr int kBoxBlock = 1024;  // largest block size of a kernel that calls box_accumulate_block

// order-preserving map of doubles to uint64 (so that integer atomic min/max order doubles)
__device__ __forceinline__ unsigned long long ord_enc(double v) {
  unsigned long long u = (unsigned long long)__double_as_longlong(v);
  return (u & 0x8000000000000000ull) ? ~u : (u | 0x8000000000000000ull);
}

__device__ __forceinline__ double ord_dec(unsigned long long u) {
  u = (u & 0x8000000000000000ull) ? (u & 0x7fffffffffffffffull) : ~u;
  return __longlong_as_double((long long)u);
}

// B-spline stencil along one axis: base node and S+1 weights.  CIC (S = 1): i = floor(u),
// f = u - i, weights (1 - f, f) on (i, i+1).  TSC (S = 2): i = floor(u + 1/2), d = u - i,
// weights (1/2 (1/2 - d)^2, 3/4 - d^2, 1/2 (1/2 + d)^2) on (i-1, i, i+1).  The base is
// clamped into the grid so that no input can address memory outside it (a valid geometry
// never needs the clamp).
template <int S>
__device__ __forceinline__ int stencil(double u, int n, double* w) {
  if constexpr (S == 1) {
    double i = floor(u);
    double f = u - i;
    w[0] = 1.0 - f;
    w[1] = f;
    int b = (int)i;
    b = b < 0 ? 0 : (b > n - 2 ? n - 2 : b);
    return b;
  } else {
    double i = floor(u + 0.5);
    double d = u - i;
    double a = 0.5 - d, c = 0.5 + d;
    w[0] = 0.5 * (a * a);
    w[1] = 0.75 - d * d;
    w[2] = 0.5 * (c * c);
    int b = (int)i - 1;
    b = b < 0 ? 0 : (b > n - 3 ? n - 3 : b);
    return b;
  }
}

// One half of a slice's linear map on the phase-space point v (rows x, px, y, py, z, delta).
__device__ __forceinline__ void apply_half(const HalfMap& h, double v[6], double inv_g2) {
  if (h.type == kHalfMatrix) {
    const double x = v[0], px = v[1], y = v[2], py = v[3];
    v[0] = h.mx[0] * x + h.mx[1] * px;
    v[1] = h.mx[2] * x + h.mx[3] * px;
    v[2] = h.my[0] * y + h.my[1] * py;
    v[3] = h.my[2] * y + h.my[3] * py;
    v[4] = v[4] + h.mz * v[5] * inv_g2;
  } else {
    if (h.type == kHalfThinDrift) {
      v[1] = v[1] - h.k * v[0];
      v[3] = v[3] + h.k * v[2];
    }
    v[0] = v[0] + h.ell * v[1];
    v[2] = v[2] + h.ell * v[3];
    v[4] = v[4] + h.ell * v[5] * inv_g2;
  }
}

// The 2x2 matrix of a half map on one transverse plane (0: x, px; 1: y, py), row-major, and
// (return value) its longitudinal coefficient c in z += c delta / gamma^2.  A thin slice's half
// map kicks first and drifts after: px -= k x, then x += l px gives ((1 - l k, l), (-k, 1)); the
// y plane has the opposite sign of k.
__device__ __forceinline__ double half_plane_matrix(const HalfMap& h, int plane, double m[4]) {
  if (h.type == kHalfMatrix) {
    const double* src = plane ? h.my : h.mx;
    for (int q = 0; q < 4; ++q) m[q] = src[q];
    return h.mz;
  }
  const double k = h.type == kHalfThinDrift ? (plane ? -h.k : h.k) : 0.0;
  m[0] = 1.0 - h.ell * k;
  m[1] = h.ell;
  m[2] = -k;
  m[3] = 1.0;
  return h.ell;
}

// The linear map "a, then b" (b_used false: a alone) as one matrix-type half map: the product of
// the two matrices per plane and the sum of the longitudinal coefficients.
__device__ __forceinline__ HalfMap half_product(const HalfMap& a, const HalfMap& b, bool b_used) {
  HalfMap r;
  r.type = kHalfMatrix;
  r.pad = 0;
  r.k = 0.0;
  r.ell = 0.0;
  double ma[4], mb[4];
  r.mz = half_plane_matrix(a, 0, ma);
  double* dst[2] = {r.mx, r.my};
  for (int plane = 0; plane < 2; ++plane) {
    half_plane_matrix(a, plane, ma);
    double* m = dst[plane];
    if (!b_used) {
      for (int q = 0; q < 4; ++q) m[q] = ma[q];
      continue;
    }
    half_plane_matrix(b, plane, mb);
    m[0] = mb[0] * ma[0] + mb[1] * ma[2];
    m[1] = mb[0] * ma[1] + mb[1] * ma[3];
    m[2] = mb[2] * ma[0] + mb[3] * ma[2];
    m[3] = mb[2] * ma[1] + mb[3] * ma[3];
  }
  if (b_used) r.mz += half_plane_matrix(b, 0, mb);
  return r;
}

// apply_half for a matrix-type map, without the branch on the type
__device__ __forceinline__ void apply_matrix(const HalfMap& h, double v[6], double inv_g2) {
  const double x = v[0], px = v[1], y = v[2], py = v[3];
  v[0] = h.mx[0] * x + h.mx[1] * px;
  v[1] = h.mx[2] * x + h.mx[3] * px;
  v[2] = h.my[0] * y + h.my[1] * py;
  v[3] = h.my[2] * y + h.my[3] * py;
  v[4] = v[4] + h.mz * v[5] * inv_g2;
}

// Transpose of apply_half on an adjoint vector lm (rows as v): the transposed matrices per
// plane and the transposed longitudinal drift; for a thin slice's first half the transposed
// drift, then the transposed thin quad.
__device__ __forceinline__ void apply_half_T(const HalfMap& h, double lm[6], double inv_g2) {
  if (h.type == kHalfMatrix) {
    const double lx = lm[0], lpx = lm[1], ly = lm[2], lpy = lm[3];
    lm[0] = h.mx[0] * lx + h.mx[2] * lpx;
    lm[1] = h.mx[1] * lx + h.mx[3] * lpx;
    lm[2] = h.my[0] * ly + h.my[2] * lpy;
    lm[3] = h.my[1] * ly + h.my[3] * lpy;
    lm[5] = lm[5] + h.mz * lm[4] * inv_g2;
  } else {
    lm[1] = lm[1] + h.ell * lm[0];
    lm[3] = lm[3] + h.ell * lm[2];
    lm[5] = lm[5] + h.ell * lm[4] * inv_g2;
    if (h.type == kHalfThinDrift) {
      lm[0] = lm[0] - h.k * lm[1];
      lm[2] = lm[2] + h.k * lm[3];
    }
  }
}

// Block-wide min/max of x, y, z, then one atomic per block and axis.
__device__ __forceinline__ void box_accumulate_block(double lo[3], double hi[3], bool bad, Box* box) {
  __shared__ double slo[3][kBoxBlock / 64], shi[3][kBoxBlock / 64];
  __shared__ int sbad;
  if (threadIdx.x == 0) sbad = 0;
  __syncthreads();
  for (int a = 0; a < 3; ++a) {
    for (int off = 32; off > 0; off >>= 1) {
      lo[a] = fmin(lo[a], __shfl_xor(lo[a], off));
      hi[a] = fmax(hi[a], __shfl_xor(hi[a], off));
    }
  }
  int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0)
    for (int a = 0; a < 3; ++a) {
      slo[a][wv] = lo[a];
      shi[a][wv] = hi[a];
    }
  if (bad) sbad = 1;
  __syncthreads();
  if (threadIdx.x < 3) {
    int a = threadIdx.x;
    double l = slo[a][0], h = shi[a][0];
    for (int q = 1; q < (int)(blockDim.x + 63) / 64; ++q) {
      l = fmin(l, slo[a][q]);
      h = fmax(h, shi[a][q]);
    }
    if (l <= h) {
      atomicMin(&box->mn[a], ord_enc(l));
      atomicMax(&box->mx[a], ord_enc(h));
    }
  }
  if (threadIdx.x == 0 && sbad) atomicOr(&box->nonfinite, 1u);
}

}  // namespace pic
