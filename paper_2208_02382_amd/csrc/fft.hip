// Free-space Poisson solve by Hockney's zero-padded FFT convolution (padded lengths M_a = 2 n_a),
// with a hand-written FFT built from LDS radix-4/2/3 stages.
//
// Green spectrum.  The cyclic Green array is real and even along every axis, so its DFT is real
// and even: Ghat(k) depends on (fold(kx), fold(ky), fold(kz)) only, fold(k) = min(k, M - k).
// It is computed on the (n_x+1)(n_y+1)(n_z+1) cell averages by three even-real DFT passes (one
// per axis; two real lines ride in one complex FFT of the even extension), in float64, then
// scaled by 1/(4 pi eps0 Mx My Mz) and stored in the grid's precision.
//
// Solve, on the half spectrum W[Mz][My][Kx] (Kx = n_x + 1):
//   r2c_x   real charge rows (y < n_y, z < n_z) -> half spectra, through a complex FFT of length
//           n_x of the even/odd-packed row and the standard split;
//   c2c y   forward along y for the planes z < n_z only (the others are zero);
//   zconv   along z: forward FFT of the n_z non-zero inputs, product with Ghat, inverse FFT, and
//           only the n_z + 2 output rows on nodes -1..n_z are written back;
//   c2c y   inverse along y for those rows, writing the n_y + 2 rows on nodes -1..n_y;
//   c2r_x   inverse real transform of those rows, writing phi on nodes -1..n_x directly.
// The field is then E' = -grad phi by centred differences (k_grad).
//
// FFT engine: a workgroup holds LB lines of length L in LDS (LB L <= 4096 complex values,
// at most 64 KB) and runs a Stockham self-sorting decimation-in-time FFT (Govindaraju et al.,
// SC'08 formulation) in place: each stage reads its butterfly inputs to registers, barriers,
// writes the outputs.  Lines along y and z are batched along x, so every row load is a run of
// LB consecutive complex values.  Twiddles come from a per-axis table exp(-2 pi i t/M) computed
// with sincospi; a half-length transform reads every second entry.
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
__device__ __forceinline__ Cx<T> cconj(Cx<T> a) { return {a.x, -a.y}; }

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

constexpr int kLdsElems = 4096;  // complex values per workgroup (64 KB for complex double)

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
    Cx<T> jt3 = DIR < 0 ? Cx<T>{t3.y, -t3.x} : Cx<T>{-t3.y, t3.x};  // -i t3 or +i t3
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

// In-place LDS FFT of LB lines of length ax.M (line l at buf[l M]).  Twiddle exp(-2 pi i t/M)
// is tw[t * tws] (tws = 2 when the table belongs to a transform twice as long).  Requires
// blockDim.x >= LB M / 4.  Ends with a barrier.
template <typename T, int DIR>
__device__ void fft_lds(Cx<T>* buf, int LB, const FftAxis& ax,
                        const typename TwT<T>::type* __restrict__ tw, int tws) {
  const int M = ax.M;
  const int NT = blockDim.x;
  const int tid = threadIdx.x;
  int Ns = 1;
  for (int s = 0; s < ax.nrad; ++s) {
    const int R = ax.rad[s];
    const int MR = M / R;
    const int nbf = LB * MR;
    Cx<T> v[2][4];
    int ob[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int bf = tid + q * NT;
      ob[q] = -1;
      if (bf < nbf) {
        const int l = bf / MR, j = bf - l * MR;
        const int k = j % Ns;
        const Cx<T>* src = buf + l * M + j;
        const int tstep = k * (M / (Ns * R)) * tws;
        for (int r = 0; r < R; ++r) {
          Cx<T> a = src[r * MR];
          if (r && tstep) {
            const auto w = tw[r * tstep];
            a = cmul(a, Cx<T>{(T)w.x, DIR < 0 ? (T)w.y : (T)-w.y});
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
}

// cyclic index of the ghost-inclusive position p = 0..n+1 (node p - 1): M - 1 for p = 0
__device__ __forceinline__ int ghost_src(int p, int M) { return p == 0 ? M - 1 : p - 1; }
__device__ __forceinline__ int fold(int k, int M) { return k <= M / 2 ? k : M - k; }

// ------------------------------------------------------------------------------ Green spectrum

// Even-real DFT along one axis of the float64 array gd[(k (ny+1) + j)(nx+1) + i] in place:
// line values g_0..g_n are extended to length M = 2n by g_t = g_{M-t}, transformed, and the
// real outputs k = 0..n stored.  Complex line c carries real lines a = 2c (real part) and
// a = 2c + 1 (imaginary part); line a starts at a*sa + b*sb, elements at stride st.
__global__ __launch_bounds__(1024) void k_green_even_dft(double* __restrict__ gd, FftAxis ax,
                                                         const double2* __restrict__ tw,
                                                         int64_t st, int64_t sa, int64_t sb,
                                                         int na, int LB) {
  extern __shared__ unsigned char smem_raw[];
  Cx<double>* buf = reinterpret_cast<Cx<double>*>(smem_raw);
  const int M = ax.M, n = M / 2;
  const int c0 = blockIdx.x * LB;  // first complex line of this block
  double* base = gd + (int64_t)blockIdx.y * sb;
  for (int idx = threadIdx.x; idx < LB * M; idx += blockDim.x) {
    const int p = idx / LB, l = idx - p * LB;  // consecutive threads: consecutive lines
    const int t = p <= n ? p : M - p;
    const int a0 = 2 * (c0 + l), a1 = a0 + 1;
    double re = a0 < na ? base[(int64_t)a0 * sa + (int64_t)t * st] : 0.0;
    double im = a1 < na ? base[(int64_t)a1 * sa + (int64_t)t * st] : 0.0;
    buf[l * M + p] = Cx<double>{re, im};
  }
  __syncthreads();
  fft_lds<double, -1>(buf, LB, ax, tw, 1);
  for (int idx = threadIdx.x; idx < LB * (n + 1); idx += blockDim.x) {
    const int p = idx / LB, l = idx - p * LB;
    const int a0 = 2 * (c0 + l), a1 = a0 + 1;
    const Cx<double> v = buf[l * M + p];
    if (a0 < na) base[(int64_t)a0 * sa + (int64_t)p * st] = v.x;
    if (a1 < na) base[(int64_t)a1 * sa + (int64_t)p * st] = v.y;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_green_finish(const Geom* __restrict__ g,
                                                      const double* __restrict__ gd,
                                                      T* __restrict__ gh, int64_t total,
                                                      double scale) {
  if (g->status) return;
  for (int64_t t = blockIdx.x * 256ll + threadIdx.x; t < total; t += (int64_t)gridDim.x * 256)
    gh[t] = (T)(gd[t] * scale);
}

// ------------------------------------------------------------------------------ solve passes

// Forward real transform of the charge rows: row (y, z) of rho (length n_x, zero-padded to
// M_x = 2 n_x) -> W[z][y][0..n_x].  Packed z_j = rho_{2j} + i rho_{2j+1}, j < n_x, complex FFT
// of length n_x (ax), then X_k = E_k + W^k O_k, E_k = (Z_k + conj Z_{n-k})/2,
// O_k = (Z_k - conj Z_{n-k})/(2i), W = exp(-2 pi i / M_x), k = 0..n_x.
template <typename T>
__global__ __launch_bounds__(1024) void k_r2c_x(const Geom* __restrict__ g,
                                                const T* __restrict__ rho, Cx<T>* __restrict__ W,
                                                FftAxis ax, const typename TwT<T>::type* __restrict__ tw,
                                                int nx, int ny, int Kx, int My, int LB) {
  extern __shared__ unsigned char smem_raw[];
  Cx<T>* buf = reinterpret_cast<Cx<T>*>(smem_raw);
  if (g->status) return;
  const int H = ax.M;  // = nx
  const int y0 = blockIdx.x * LB, z = blockIdx.y;
  const int nl = min(LB, ny - y0);
  const T* src = rho + ((int64_t)z * ny + y0) * nx;
  for (int idx = threadIdx.x; idx < LB * H; idx += blockDim.x) {
    const int l = idx / H, j = idx - l * H;
    Cx<T> v = {0, 0};
    if (l < nl && 2 * j < nx) {
      v.x = src[(int64_t)l * nx + 2 * j];
      v.y = 2 * j + 1 < nx ? src[(int64_t)l * nx + 2 * j + 1] : T(0);
    }
    buf[l * H + j] = v;
  }
  __syncthreads();
  fft_lds<T, -1>(buf, LB, ax, tw, 2);
  Cx<T>* dst = W + ((int64_t)z * My + y0) * Kx;
  for (int idx = threadIdx.x; idx < LB * (H + 1); idx += blockDim.x) {
    const int l = idx / (H + 1), k = idx - l * (H + 1);
    if (l >= nl) continue;
    const Cx<T> zk = buf[l * H + (k % H)];
    const Cx<T> zc = cconj(buf[l * H + ((H - k) % H)]);
    const Cx<T> e = {(T)0.5 * (zk.x + zc.x), (T)0.5 * (zk.y + zc.y)};
    const Cx<T> dif = csub(zk, zc);
    const Cx<T> o = {(T)0.5 * dif.y, (T)-0.5 * dif.x};  // dif / (2i)
    const auto w = tw[k];                              // exp(-2 pi i k / M_x)
    dst[(int64_t)l * Kx + k] = cadd(e, cmul(Cx<T>{(T)w.x, (T)w.y}, o));
  }
}

// Complex line FFT in place along y (element stride Kx) for lines a = kx (stride 1) and
// b = plane (stride My Kx).  Inputs p < n_in are read (the rest are zero); GHOST stores only the
// positions q = 0..n+1 taken from cyclic index ghost_src(q), otherwise all M outputs.
template <typename T, int DIR, bool GHOST>
__global__ __launch_bounds__(1024) void k_c2c_y(const Geom* __restrict__ g, Cx<T>* __restrict__ W,
                                                FftAxis ax,
                                                const typename TwT<T>::type* __restrict__ tw,
                                                int Kx, int n_in, int n_ghost, int LB) {
  extern __shared__ unsigned char smem_raw[];
  Cx<T>* buf = reinterpret_cast<Cx<T>*>(smem_raw);
  if (g->status) return;
  const int M = ax.M;
  const int a0 = blockIdx.x * LB;
  const int nl = min(LB, Kx - a0);
  Cx<T>* base = W + (int64_t)blockIdx.y * M * Kx + a0;
  for (int idx = threadIdx.x; idx < LB * M; idx += blockDim.x) {
    const int p = idx / LB, l = idx - p * LB;
    Cx<T> v = {0, 0};
    if (l < nl && p < n_in) v = base[(int64_t)p * Kx + l];
    buf[l * M + p] = v;
  }
  __syncthreads();
  fft_lds<T, DIR>(buf, LB, ax, tw, 1);
  const int nout = GHOST ? n_ghost : M;
  for (int idx = threadIdx.x; idx < LB * nout; idx += blockDim.x) {
    const int q = idx / LB, l = idx - q * LB;
    if (l < nl) base[(int64_t)q * Kx + l] = buf[l * M + (GHOST ? ghost_src(q, M) : q)];
  }
}

// Along z (element stride My Kx) for lines a = kx, b = ky: forward FFT of the n_z non-zero
// inputs, product with Ghat(fold kz, fold ky, kx) (gh[(fz (ny+1) + fy)(nx+1) + kx]), inverse
// FFT, and the n_z + 2 ghost-inclusive rows written back in place.
template <typename T>
__global__ __launch_bounds__(1024) void k_zconv(const Geom* __restrict__ g, Cx<T>* __restrict__ W,
                                                const T* __restrict__ gh, FftAxis ax,
                                                const typename TwT<T>::type* __restrict__ tw,
                                                int Kx, int My, int ny, int nz, int LB) {
  extern __shared__ unsigned char smem_raw[];
  Cx<T>* buf = reinterpret_cast<Cx<T>*>(smem_raw);
  if (g->status) return;
  const int M = ax.M;
  const int a0 = blockIdx.x * LB, ky = blockIdx.y;
  const int nl = min(LB, Kx - a0);
  const int64_t sz = (int64_t)My * Kx;
  Cx<T>* base = W + (int64_t)ky * Kx + a0;
  for (int idx = threadIdx.x; idx < LB * M; idx += blockDim.x) {
    const int p = idx / LB, l = idx - p * LB;
    Cx<T> v = {0, 0};
    if (l < nl && p < nz) v = base[(int64_t)p * sz + l];
    buf[l * M + p] = v;
  }
  __syncthreads();
  fft_lds<T, -1>(buf, LB, ax, tw, 1);
  const int fy = fold(ky, My);
  const T* grow = gh + (int64_t)fy * Kx + a0;
  const int64_t gplane = (int64_t)(ny + 1) * Kx;
  for (int idx = threadIdx.x; idx < LB * M; idx += blockDim.x) {
    const int p = idx / LB, l = idx - p * LB;
    if (l < nl) {
      const T s = grow[(int64_t)fold(p, M) * gplane + l];
      Cx<T> v = buf[l * M + p];
      buf[l * M + p] = Cx<T>{v.x * s, v.y * s};
    }
  }
  __syncthreads();
  fft_lds<T, +1>(buf, LB, ax, tw, 1);
  for (int idx = threadIdx.x; idx < LB * (nz + 2); idx += blockDim.x) {
    const int q = idx / LB, l = idx - q * LB;
    if (l < nl) base[(int64_t)q * sz + l] = buf[l * M + ghost_src(q, M)];
  }
}

// Inverse real transform of the rows (yy, zz) of W (yy < ny + 2, zz < nz + 2), writing phi on
// x-nodes -1..n_x: Z_k = (X_k + conj X_{n-k}) + i exp(+2 pi i k/M_x)(X_k - conj X_{n-k}),
// k < n = n_x, inverse complex FFT of length n_x, x_{2j} = Re z_j, x_{2j+1} = Im z_j.
template <typename T>
__global__ __launch_bounds__(1024) void k_c2r_x(const Geom* __restrict__ g,
                                                const Cx<T>* __restrict__ W, T* __restrict__ phi,
                                                FftAxis ax,
                                                const typename TwT<T>::type* __restrict__ tw,
                                                int nx, int ny, int Kx, int My, int LB) {
  extern __shared__ unsigned char smem_raw[];
  Cx<T>* buf = reinterpret_cast<Cx<T>*>(smem_raw);
  if (g->status) return;
  const int H = ax.M;  // = nx
  const int M = 2 * H;
  const int py = ny + 2;
  const int r0 = blockIdx.x * LB, zz = blockIdx.y;
  const int nl = min(LB, py - r0);
  const Cx<T>* src = W + ((int64_t)zz * My + r0) * Kx;
  for (int idx = threadIdx.x; idx < LB * H; idx += blockDim.x) {
    const int l = idx / H, k = idx - l * H;
    Cx<T> v = {0, 0};
    if (l < nl) {
      const Cx<T> xk = src[(int64_t)l * Kx + k];
      const Cx<T> xc = cconj(src[(int64_t)l * Kx + (H - k)]);
      const auto w = tw[k];
      const Cx<T> winv = {(T)w.x, (T)-w.y};  // exp(+2 pi i k / M_x)
      const Cx<T> d = cmul(winv, csub(xk, xc));
      v = cadd(cadd(xk, xc), Cx<T>{-d.y, d.x});  // + i d
    }
    buf[l * H + k] = v;
  }
  __syncthreads();
  fft_lds<T, +1>(buf, LB, ax, tw, 2);
  const int px = nx + 2;
  T* dst = phi + ((int64_t)zz * py + r0) * px;
  for (int idx = threadIdx.x; idx < LB * px; idx += blockDim.x) {
    const int l = idx / px, q = idx - l * px;
    if (l < nl) {
      const int t = ghost_src(q, M);
      const Cx<T> zj = buf[l * H + (t >> 1)];
      dst[(int64_t)l * px + q] = (t & 1) ? zj.y : zj.x;
    }
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

__global__ void k_twiddles(double2* tw, float2* twf, int M) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= M) return;
  double s, c;
  sincospi(2.0 * (double)t / (double)M, &s, &c);
  tw[t] = make_double2(c, -s);
  twf[t] = make_float2((float)c, (float)-s);
}

int grid_for(int64_t total) {
  int64_t b = (total + 255) / 256;
  if (b > 16384) b = 16384;
  return (int)(b < 1 ? 1 : b);
}

// lines per workgroup and threads for transforms of length L over `lines` lines
void shape_for(int L, int lines, int* LB, int* NT) {
  int lb = kLdsElems / L;
  if (lb < 1) lb = 1;
  if (lb > lines) lb = lines;
  int nt = (lb * L + 3) / 4;
  nt = ((nt + 63) / 64) * 64;
  if (nt > 1024) nt = 1024;
  if (nt < 64) nt = 64;
  *LB = lb;
  *NT = nt;
}

template <typename T>
const typename TwT<T>::type* table(const FftPlan& p, int a);
template <>
const double2* table<double>(const FftPlan& p, int a) { return p.tw[a]; }
template <>
const float2* table<float>(const FftPlan& p, int a) { return p.twf[a]; }

}  // namespace

hipError_t launch_twiddles(double2* tw, float2* twf, int M, hipStream_t s) {
  hipLaunchKernelGGL(k_twiddles, dim3((M + 255) / 256), dim3(256), 0, s, tw, twf, M);
  return hipGetLastError();
}

#define PIC_TRY(x)                   \
  do {                               \
    hipError_t e_ = (x);             \
    if (e_ != hipSuccess) return e_; \
  } while (0)

template <typename T>
hipError_t launch_green_spectrum(const Geom* g, const FftPlan& p, int nx, int ny, int nz,
                                 double2* corners, double* gd, T* gh, hipStream_t s) {
  PIC_TRY(launch_igf_corners(g, nx, ny, nz, corners, s));
  PIC_TRY(launch_igf_cells(g, nx, ny, nz, corners, gd, s));
  const int ex = nx + 1, ey = ny + 1, ez = nz + 1;
  // (axis, element stride, line stride a, plane stride b, lines a, planes b)
  const int64_t cfg[3][5] = {{1, ex, (int64_t)ex * ey, ey, ez},
                             {ex, 1, (int64_t)ex * ey, ex, ez},
                             {(int64_t)ex * ey, 1, 0, (int64_t)ex * ey, 1}};
  for (int a = 0; a < 3; ++a) {
    const int na = (int)cfg[a][3];
    const int ncx = (na + 1) / 2;  // complex lines (two real lines each)
    int LB, NT;
    shape_for(p.full[a].M, ncx, &LB, &NT);
    dim3 grid((ncx + LB - 1) / LB, (unsigned)cfg[a][4]);
    size_t lds = (size_t)LB * p.full[a].M * sizeof(Cx<double>);
    hipLaunchKernelGGL(k_green_even_dft, grid, dim3(NT), lds, s, gd, p.full[a], p.tw[a],
                       cfg[a][0], cfg[a][1], cfg[a][2], na, LB);
    PIC_TRY(hipGetLastError());
  }
  const int64_t total = (int64_t)ex * ey * ez;
  const double scale =
      1.0 / (4.0 * 3.14159265358979323846 * 8.8541878128e-12 * (8.0 * nx * ny * nz));
  hipLaunchKernelGGL((k_green_finish<T>), dim3(grid_for(total)), dim3(256), 0, s, g, gd, gh,
                     total, scale);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_solve(const Geom* g, const FftPlan& p, int nx, int ny, int nz, const T* rho,
                        void* Wv, const T* gh, T* phi, T* E, hipStream_t s) {
  Cx<T>* W = (Cx<T>*)Wv;
  const int My = 2 * ny, Kx = nx + 1;
  int LB, NT;
  size_t lds;
  // r2c along x: rows (y < ny, z < nz)
  shape_for(p.half_x.M, ny, &LB, &NT);
  lds = (size_t)LB * p.half_x.M * sizeof(Cx<T>);
  hipLaunchKernelGGL((k_r2c_x<T>), dim3((ny + LB - 1) / LB, nz), dim3(NT), lds, s, g, rho, W,
                     p.half_x, table<T>(p, 0), nx, ny, Kx, My, LB);
  PIC_TRY(hipGetLastError());
  // forward along y, planes z < nz
  shape_for(p.full[1].M, Kx, &LB, &NT);
  lds = (size_t)LB * p.full[1].M * sizeof(Cx<T>);
  hipLaunchKernelGGL((k_c2c_y<T, -1, false>), dim3((Kx + LB - 1) / LB, nz), dim3(NT), lds, s, g,
                     W, p.full[1], table<T>(p, 1), Kx, ny, 0, LB);
  PIC_TRY(hipGetLastError());
  // z: forward, product with the Green spectrum, inverse; rows on nodes -1..nz
  shape_for(p.full[2].M, Kx, &LB, &NT);
  lds = (size_t)LB * p.full[2].M * sizeof(Cx<T>);
  hipLaunchKernelGGL((k_zconv<T>), dim3((Kx + LB - 1) / LB, My), dim3(NT), lds, s, g, W, gh,
                     p.full[2], table<T>(p, 2), Kx, My, ny, nz, LB);
  PIC_TRY(hipGetLastError());
  // inverse along y for the nz + 2 rows; rows on nodes -1..ny
  shape_for(p.full[1].M, Kx, &LB, &NT);
  lds = (size_t)LB * p.full[1].M * sizeof(Cx<T>);
  hipLaunchKernelGGL((k_c2c_y<T, +1, true>), dim3((Kx + LB - 1) / LB, nz + 2), dim3(NT), lds, s,
                     g, W, p.full[1], table<T>(p, 1), Kx, My, ny + 2, LB);
  PIC_TRY(hipGetLastError());
  // c2r along x for the (ny + 2)(nz + 2) rows, phi on nodes -1..nx
  shape_for(p.half_x.M, ny + 2, &LB, &NT);
  lds = (size_t)LB * p.half_x.M * sizeof(Cx<T>);
  hipLaunchKernelGGL((k_c2r_x<T>), dim3((ny + 2 + LB - 1) / LB, nz + 2), dim3(NT), lds, s, g, W,
                     phi, p.half_x, table<T>(p, 0), nx, ny, Kx, My, LB);
  PIC_TRY(hipGetLastError());
  const int64_t ng = (int64_t)nx * ny * nz;
  hipLaunchKernelGGL((k_grad<T>), dim3(grid_for(ng)), dim3(256), 0, s, g, phi, E, nx, ny, nz);
  return hipGetLastError();
}

template hipError_t launch_green_spectrum<double>(const Geom*, const FftPlan&, int, int, int,
                                                  double2*, double*, double*, hipStream_t);
template hipError_t launch_green_spectrum<float>(const Geom*, const FftPlan&, int, int, int,
                                                 double2*, double*, float*, hipStream_t);
template hipError_t launch_solve<double>(const Geom*, const FftPlan&, int, int, int,
                                         const double*, void*, const double*, double*, double*,
                                         hipStream_t);
template hipError_t launch_solve<float>(const Geom*, const FftPlan&, int, int, int, const float*,
                                        void*, const float*, float*, float*, hipStream_t);

}  // namespace pic
