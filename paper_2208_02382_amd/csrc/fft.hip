// Free-space Poisson solve by Hockney's zero-padded FFT convolution, with a hand-written
// 3-D FFT built from LDS radix-4/2/3 stages.
//
// The charge array (nz, ny, nx) is embedded in a cyclic (2nz, 2ny, 2nx) complex array W; the
// forward transform of W times the real spectrum of the even-symmetrically placed integrated
// Green's function, transformed back, equals the free-space sum on nodes -1..n_a of each axis
// (the cyclic images fall outside those nodes).  The field is -grad phi by centred differences.
//
// FFT: every pass transforms a batch of lines of length M along one axis.  A workgroup stages
// LB = 2048/M lines in LDS (lines along x are contiguous; along y and z the LB lines are
// adjacent in x, so each row load is an LB-element contiguous run), runs the stages of a
// Stockham self-sorting decimation-in-time FFT (Govindaraju et al., SC'08 formulation) in
// place in LDS -- each stage reads its butterfly inputs to registers, barriers, writes the
// outputs -- and writes the lines back.  Twiddles come from a per-axis table
// exp(-2 pi i t/M) computed with sincospi.  Zero inputs past `n_in` are not read (the zero
// padding) and lines known to be zero are not launched.
#include "internal.hpp"

namespace pic {

namespace {

template <typename T>
struct Cx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ Cx<T> cmul(Cx<T> a, Cx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ Cx<T> cadd(Cx<T> a, Cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ Cx<T> csub(Cx<T> a, Cx<T> b) { return {a.x - b.x, a.y - b.y}; }

template <typename T>
struct TwT;
template <>
struct TwT<double> {
  using type = double2;
};
template <>
struct TwT<float> {
  using type = float2;
};

constexpr int kElems = 2048;  // LDS elements per workgroup (32 KB for complex double)

struct AxisArgs {
  int M;
  int nrad;
  int rad[12];
};

// Radix-R DFT in registers; DIR = -1 forward, +1 inverse (no scaling).
template <typename T, int DIR>
__device__ __forceinline__ void dft(Cx<T>* v, int R) {
  if (R == 2) {
    Cx<T> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if (R == 4) {
    Cx<T> t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    Cx<T> t2 = cadd(v[1], v[3]), t3 = csub(v[1], v[3]);
    // multiply t3 by -i (forward) or +i (inverse)
    Cx<T> jt3 = DIR < 0 ? Cx<T>{t3.y, -t3.x} : Cx<T>{-t3.y, t3.x};
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, jt3);
    v[3] = csub(t1, jt3);
  } else {  // R == 3
    const T s3 = (T)(DIR < 0 ? -0.86602540378443864676 : 0.86602540378443864676);
    Cx<T> a0 = v[0], a1 = v[1], a2 = v[2];
    Cx<T> sum = cadd(a1, a2), dif = csub(a1, a2);
    Cx<T> m = {a0.x - (T)0.5 * sum.x, a0.y - (T)0.5 * sum.y};
    Cx<T> jd = {-s3 * dif.y, s3 * dif.x};  // i s3 (a1 - a2)
    v[0] = cadd(a0, sum);
    v[1] = cadd(m, jd);
    v[2] = csub(m, jd);
  }
}

// One pass: lines a = 0..na-1 (stride sa), b = blockIdx.y (stride sb), element stride st.
template <typename T, int DIR>
__global__ __launch_bounds__(512) void k_fft_lines(Cx<T>* __restrict__ data, AxisArgs ax,
                                                   const typename TwT<T>::type* __restrict__ tw,
                                                   int64_t st, int64_t sa, int64_t sb, int na,
                                                   int n_in, int LB) {
  extern __shared__ unsigned char smem_raw[];
  Cx<T>* buf = reinterpret_cast<Cx<T>*>(smem_raw);
  const int M = ax.M;
  const int NT = blockDim.x;
  const int tid = threadIdx.x;
  const int a0 = blockIdx.x * LB;
  const int nl = min(LB, na - a0);
  Cx<T>* base = data + (int64_t)blockIdx.y * sb + (int64_t)a0 * sa;
  const int total = LB * M;
  // load (zero padding beyond n_in and beyond the last line)
  if (st == 1) {
    for (int idx = tid; idx < total; idx += NT) {
      int l = idx / M, p = idx - l * M;
      Cx<T> v = {0, 0};
      if (l < nl && p < n_in) v = base[(int64_t)l * sa + p];
      buf[l * M + p] = v;
    }
  } else {
    for (int idx = tid; idx < total; idx += NT) {
      int p = idx / LB, l = idx - p * LB;
      Cx<T> v = {0, 0};
      if (l < nl && p < n_in) v = base[(int64_t)l * sa + (int64_t)p * st];
      buf[l * M + p] = v;
    }
  }
  __syncthreads();
  int Ns = 1;
  for (int s = 0; s < ax.nrad; ++s) {
    const int R = ax.rad[s];
    const int MR = M / R;
    const int nbf = LB * MR;
    Cx<T> v[2][4];
    int ob[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      int bf = tid + q * NT;
      ob[q] = -1;
      if (bf < nbf) {
        int l = bf / MR, j = bf - l * MR;
        int k = j % Ns;
        const Cx<T>* src = buf + l * M + j;
        int tstep = k * (M / (Ns * R));
        for (int r = 0; r < R; ++r) {
          Cx<T> a = src[r * MR];
          if (r && tstep) {
            auto w = tw[r * tstep];
            Cx<T> wc = {w.x, DIR < 0 ? w.y : -w.y};
            a = cmul(a, wc);
          }
          v[q][r] = a;
        }
        dft<T, DIR>(v[q], R);
        ob[q] = l * M + (j / Ns) * Ns * R + k;
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 2; ++q)
      if (ob[q] >= 0)
        for (int r = 0; r < R; ++r) buf[ob[q] + r * Ns] = v[q][r];
    __syncthreads();
    Ns *= R;
  }
  // store
  if (st == 1) {
    for (int idx = tid; idx < total; idx += NT) {
      int l = idx / M, p = idx - l * M;
      if (l < nl) base[(int64_t)l * sa + p] = buf[l * M + p];
    }
  } else {
    for (int idx = tid; idx < total; idx += NT) {
      int p = idx / LB, l = idx - p * LB;
      if (l < nl) base[(int64_t)l * sa + (int64_t)p * st] = buf[l * M + p];
    }
  }
}

__global__ void k_twiddles(double2* tw, float2* twf, int M) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= M) return;
  double s, c;
  sincospi(2.0 * (double)t / (double)M, &s, &c);
  tw[t] = make_double2(c, -s);
  twf[t] = make_float2((float)c, (float)-s);
}

// W = charge on (z < nz, y < ny, x < nx), zero elsewhere
template <typename T>
__global__ __launch_bounds__(256) void k_pad(const Geom* __restrict__ g, const T* __restrict__ rho,
                                             Cx<T>* __restrict__ W, int nx, int ny, int nz) {
  if (g->status) return;
  const int Mx = 2 * nx, My = 2 * ny;
  const int64_t total = (int64_t)Mx * My * 2 * nz;
  for (int64_t t = blockIdx.x * 256ll + threadIdx.x; t < total; t += (int64_t)gridDim.x * 256) {
    int x = (int)(t % Mx), y = (int)((t / Mx) % My), z = (int)(t / ((int64_t)Mx * My));
    T v = 0;
    if (x < nx && y < ny && z < nz) v = rho[((int64_t)z * ny + y) * nx + x];
    W[t] = Cx<T>{v, 0};
  }
}

// Gh = Re(W) * scale, scale = 1/(4 pi eps0 M^3): the Green spectrum with the solve constants
template <typename T>
__global__ __launch_bounds__(256) void k_green_extract(const Geom* __restrict__ g,
                                                       const Cx<T>* __restrict__ W,
                                                       T* __restrict__ Gh, int64_t total,
                                                       double scale) {
  if (g->status) return;
  for (int64_t t = blockIdx.x * 256ll + threadIdx.x; t < total; t += (int64_t)gridDim.x * 256)
    Gh[t] = (T)((double)W[t].x * scale);
}

template <typename T>
__global__ __launch_bounds__(256) void k_mul(const Geom* __restrict__ g, Cx<T>* __restrict__ W,
                                             const T* __restrict__ Gh, int64_t total) {
  if (g->status) return;
  for (int64_t t = blockIdx.x * 256ll + threadIdx.x; t < total; t += (int64_t)gridDim.x * 256) {
    Cx<T> w = W[t];
    T s = Gh[t];
    W[t] = Cx<T>{w.x * s, w.y * s};
  }
}

// phi[(kz (ny+2) + ky)(nx+2) + kx] = Re W at cyclic index (k == 0 ? M-1 : k-1) per axis,
// i.e. phi on nodes -1..n_a
template <typename T>
__global__ __launch_bounds__(256) void k_extract_phi(const Geom* __restrict__ g,
                                                     const Cx<T>* __restrict__ W,
                                                     T* __restrict__ phi, int nx, int ny,
                                                     int nz) {
  if (g->status) return;
  const int px = nx + 2, py = ny + 2, pz = nz + 2;
  const int Mx = 2 * nx, My = 2 * ny, Mz = 2 * nz;
  const int64_t total = (int64_t)px * py * pz;
  for (int64_t t = blockIdx.x * 256ll + threadIdx.x; t < total; t += (int64_t)gridDim.x * 256) {
    int kx = (int)(t % px), ky = (int)((t / px) % py), kz = (int)(t / ((int64_t)px * py));
    int x = kx == 0 ? Mx - 1 : kx - 1;
    int y = ky == 0 ? My - 1 : ky - 1;
    int z = kz == 0 ? Mz - 1 : kz - 1;
    phi[t] = W[((int64_t)z * My + y) * Mx + x].x;
  }
}

// E'[c][k][j][i] = -(phi(n + e_c) - phi(n - e_c)) / (2 h_c), rest-frame spacings
template <typename T>
__global__ __launch_bounds__(256) void k_grad(const Geom* __restrict__ g, const T* __restrict__ phi,
                                              T* __restrict__ E, int nx, int ny, int nz) {
  if (g->status) return;
  const int px = nx + 2, py = ny + 2;
  const int64_t total = (int64_t)nx * ny * nz;
  const T cx = (T)(1.0 / (2.0 * g->h_rest[0]));
  const T cy = (T)(1.0 / (2.0 * g->h_rest[1]));
  const T cz = (T)(1.0 / (2.0 * g->h_rest[2]));
  const int64_t sy = px, sz = (int64_t)px * py;
  for (int64_t t = blockIdx.x * 256ll + threadIdx.x; t < total; t += (int64_t)gridDim.x * 256) {
    int i = (int)(t % nx), j = (int)((t / nx) % ny), k = (int)(t / ((int64_t)nx * ny));
    int64_t c = (int64_t)(k + 1) * sz + (int64_t)(j + 1) * sy + (i + 1);
    E[t] = -(phi[c + 1] - phi[c - 1]) * cx;
    E[total + t] = -(phi[c + sy] - phi[c - sy]) * cy;
    E[2 * total + t] = -(phi[c + sz] - phi[c - sz]) * cz;
  }
}

int grid_for(int64_t total) {
  int64_t b = (total + 255) / 256;
  if (b > 16384) b = 16384;
  return (int)(b < 1 ? 1 : b);
}

AxisArgs axis_args(const FftPlan& p, int a) {
  AxisArgs ax;
  ax.M = p.M[a];
  ax.nrad = p.nrad[a];
  for (int q = 0; q < 12; ++q) ax.rad[q] = p.rad[a][q];
  return ax;
}

template <typename T>
const typename TwT<T>::type* table(const FftPlan& p, int a);
template <>
const double2* table<double>(const FftPlan& p, int a) { return p.tw[a]; }
template <>
const float2* table<float>(const FftPlan& p, int a) { return p.twf[a]; }

// One batched line pass along axis `a` of the cyclic array W[Mz][My][Mx].
// Lines: along x -> (a: y < ny_lines, b: z < nz_lines); along y -> (a: x < Mx, b: z < nz_lines);
// along z -> (a: x < Mx, b: y < My).
template <typename T, int DIR>
hipError_t pass(Cx<T>* W, const FftPlan& p, int a, int lines_a, int lines_b, int n_in,
                hipStream_t s) {
  const int Mx = p.M[0], My = p.M[1];
  int64_t st, sa, sb;
  if (a == 0) {
    st = 1; sa = Mx; sb = (int64_t)Mx * My;
  } else if (a == 1) {
    st = Mx; sa = 1; sb = (int64_t)Mx * My;
  } else {
    st = (int64_t)Mx * My; sa = 1; sb = Mx;
  }
  const int M = p.M[a];
  int LB = kElems / M;
  if (LB < 1) LB = 1;
  int NT = (LB * M + 3) / 4;
  NT = ((NT + 63) / 64) * 64;
  if (NT > 512) NT = 512;
  size_t lds = (size_t)LB * M * sizeof(Cx<T>);
  dim3 grid((lines_a + LB - 1) / LB, lines_b);
  hipLaunchKernelGGL((k_fft_lines<T, DIR>), grid, dim3(NT), lds, s, W, axis_args(p, a),
                     table<T>(p, a), st, sa, sb, lines_a, n_in, LB);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_twiddles(double2* tw, float2* twf, int M, hipStream_t s) {
  hipLaunchKernelGGL(k_twiddles, dim3((M + 255) / 256), dim3(256), 0, s, tw, twf, M);
  return hipGetLastError();
}

#define PIC_TRY(x)                  \
  do {                              \
    hipError_t e_ = (x);            \
    if (e_ != hipSuccess) return e_; \
  } while (0)

template <typename T>
hipError_t launch_green_spectrum(const Geom* g, const FftPlan& p, int nx, int ny, int nz,
                                 double2* corners, void* Wv, T* Gh, hipStream_t s) {
  Cx<T>* W = (Cx<T>*)Wv;
  const int Mx = p.M[0], My = p.M[1], Mz = p.M[2];
  PIC_TRY(launch_igf_corners(g, nx, ny, nz, corners, s));
  PIC_TRY(launch_igf_place<T>(g, nx, ny, nz, corners, Wv, s));
  PIC_TRY((pass<T, -1>(W, p, 0, My, Mz, Mx, s)));
  PIC_TRY((pass<T, -1>(W, p, 1, Mx, Mz, My, s)));
  PIC_TRY((pass<T, -1>(W, p, 2, Mx, My, Mz, s)));
  const int64_t total = (int64_t)Mx * My * Mz;
  const double scale = 1.0 / (4.0 * 3.14159265358979323846 * 8.8541878128e-12 * (double)total);
  hipLaunchKernelGGL((k_green_extract<T>), dim3(grid_for(total)), dim3(256), 0, s, g, W, Gh,
                     total, scale);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_solve(const Geom* g, const FftPlan& p, int nx, int ny, int nz, const T* rho,
                        void* Wv, const T* Gh, T* phi, T* E, hipStream_t s) {
  Cx<T>* W = (Cx<T>*)Wv;
  const int Mx = p.M[0], My = p.M[1], Mz = p.M[2];
  const int64_t total = (int64_t)Mx * My * Mz;
  hipLaunchKernelGGL((k_pad<T>), dim3(grid_for(total)), dim3(256), 0, s, g, rho, W, nx, ny, nz);
  PIC_TRY(hipGetLastError());
  // forward: only lines that can be non-zero, only the first n_a inputs of each line
  PIC_TRY((pass<T, -1>(W, p, 0, ny, nz, nx, s)));
  PIC_TRY((pass<T, -1>(W, p, 1, Mx, nz, ny, s)));
  PIC_TRY((pass<T, -1>(W, p, 2, Mx, My, nz, s)));
  hipLaunchKernelGGL((k_mul<T>), dim3(grid_for(total)), dim3(256), 0, s, g, W, Gh, total);
  PIC_TRY(hipGetLastError());
  PIC_TRY((pass<T, +1>(W, p, 2, Mx, My, Mz, s)));
  PIC_TRY((pass<T, +1>(W, p, 1, Mx, Mz, My, s)));
  PIC_TRY((pass<T, +1>(W, p, 0, My, Mz, Mx, s)));
  const int64_t np = (int64_t)(nx + 2) * (ny + 2) * (nz + 2);
  hipLaunchKernelGGL((k_extract_phi<T>), dim3(grid_for(np)), dim3(256), 0, s, g, W, phi, nx, ny,
                     nz);
  PIC_TRY(hipGetLastError());
  const int64_t ng = (int64_t)nx * ny * nz;
  hipLaunchKernelGGL((k_grad<T>), dim3(grid_for(ng)), dim3(256), 0, s, g, phi, E, nx, ny, nz);
  return hipGetLastError();
}

template hipError_t launch_green_spectrum<double>(const Geom*, const FftPlan&, int, int, int,
                                                  double2*, void*, double*, hipStream_t);
template hipError_t launch_green_spectrum<float>(const Geom*, const FftPlan&, int, int, int,
                                                 double2*, void*, float*, hipStream_t);
template hipError_t launch_solve<double>(const Geom*, const FftPlan&, int, int, int,
                                         const double*, void*, const double*, double*, double*,
                                         hipStream_t);
template hipError_t launch_solve<float>(const Geom*, const FftPlan&, int, int, int, const float*,
                                        void*, const float*, float*, float*, hipStream_t);

}  // namespace pic
