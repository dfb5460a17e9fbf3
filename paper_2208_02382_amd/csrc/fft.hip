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
struct TwT;
template <>
struct TwT<double> {
  using type = double2;
};
template <>
struct TwT<float> {
  using type = float2;
};

// complex load through the native vector type (a struct copy of a conditional load otherwise
// goes through scratch memory)
template <typename T>
__device__ __forceinline__ Cx<T> ld(const Cx<T>* p) {
  const typename TwT<T>::type t = *reinterpret_cast<const typename TwT<T>::type*>(p);
  return Cx<T>{t.x, t.y};
}

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

constexpr int kLdsElems = 4096;  // complex values per workgroup (64 KB for complex double)

// Radix-R DFT in registers; DIR = -1 forward, +1 inverse (no scaling).  R is a template
// parameter so that the butterfly values stay in registers (a runtime radix makes the compiler
// place them in scratch memory).
template <typename T, int DIR, int R>
__device__ __forceinline__ void dft(Cx<T>* v) {
  if constexpr (R == 2) {
    Cx<T> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if constexpr (R == 4) {
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

// One Stockham stage of radix R over LB lines of length M (line stride M + 1): butterfly bf
// (line l, j < M/R, k = j mod Ns) reads buf[l, j + r M/R], applies the twiddles
// exp(-+2 pi i r k / (Ns R)) and the radix-R DFT, and writes buf[l, (j / Ns) Ns R + k + r Ns].
// Each thread takes up to two butterflies; inputs are read before the barrier and outputs
// written after it.
template <typename T, int DIR, int R>
__device__ __forceinline__ void fft_stage(Cx<T>* buf, int LB, int M, int Ns,
                                          const typename TwT<T>::type* tw, int tws) {
  const int MR = M / R;
  const int nbf = LB * MR;
  const int NT = blockDim.x;
  Cx<T> v[2][R];
  int ob[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int bf = threadIdx.x + q * NT;
    ob[q] = -1;
    if (bf < nbf) {
      const int l = bf / MR, j = bf - l * MR;
      const int k = j % Ns;
      const Cx<T>* src = buf + l * (M + 1) + j;
      const int tstep = k * (M / (Ns * R)) * tws;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        Cx<T> a = src[r * MR];
        if (r && tstep) {
          const auto w = tw[r * tstep];
          a = cmul(a, Cx<T>{(T)w.x, DIR < 0 ? (T)w.y : (T)-w.y});
        }
        v[q][r] = a;
      }
      dft<T, DIR, R>(v[q]);
      ob[q] = l * (M + 1) + (j / Ns) * Ns * R + k;
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 2; ++q)
    if (ob[q] >= 0) {
#pragma unroll
      for (int r = 0; r < R; ++r) buf[ob[q] + r * Ns] = v[q][r];
    }
  __syncthreads();
}

// In-place LDS FFT of LB lines of length ax.M (line l at buf[l (M + 1)]: the padding of one
// element per line spreads the transposed loads and stores of y and z lines over the LDS
// banks).  Twiddle exp(-2 pi i t/M) is tw[t * tws] (tws = 2 when the table belongs to a
// transform twice as long).  Requires blockDim.x >= LB M / 4.  Ends with a barrier.
template <typename T, int DIR>
__device__ void fft_lds(Cx<T>* buf, int LB, const FftAxis& ax, const typename TwT<T>::type* tw,
                        int tws) {
  // the planner's radix order: all factors 4, then 2, then 3 (derived from M here, so that
  // no array is indexed at run time)
  const int M = ax.M;
  int m = M, Ns = 1;
  while (m % 4 == 0) {
    fft_stage<T, DIR, 4>(buf, LB, M, Ns, tw, tws);
    Ns *= 4;
    m /= 4;
  }
  while (m % 2 == 0) {
    fft_stage<T, DIR, 2>(buf, LB, M, Ns, tw, tws);
    Ns *= 2;
    m /= 2;
  }
  while (m % 3 == 0) {
    fft_stage<T, DIR, 3>(buf, LB, M, Ns, tw, tws);
    Ns *= 3;
    m /= 3;
  }
}

// Copies `count` twiddles into LDS right after the LB lines of buf (LB (M + 1) elements), so
// that the stages read them from LDS instead of global memory; ordered before the first stage
// by the barrier that ends the caller's load phase.
template <typename T>
__device__ __forceinline__ const typename TwT<T>::type* stage_twiddles(
    Cx<T>* buf, int LB, int M, const typename TwT<T>::type* __restrict__ tw, int count) {
  auto* twl = reinterpret_cast<typename TwT<T>::type*>(buf + LB * (M + 1));
  for (int t = threadIdx.x; t < count; t += blockDim.x) twl[t] = tw[t];
  return twl;
}

// Fills the LB lines of length M in LDS (line l at buf[l (M + 1)]) from global memory, element
// p of line l from addr(p, l) where ok(p, l) holds and zero elsewhere; consecutive threads take
// consecutive lines, which are consecutive in memory.  A thread issues its loads four at a time
// before it stores any of them to LDS, the addresses of elements that are not loaded replaced by
// `safe` (any valid address) and the values by zero, so that no branch surrounds a load: a load
// inside a branch is waited for at the branch's join, which would put the latencies of a
// thread's loads one after another.
template <typename T, typename Addr, typename Ok>
__device__ __forceinline__ void load_lines(Cx<T>* buf, int LB, int M, const Cx<T>* safe,
                                           Addr addr, Ok ok) {
  const int total = LB * M, nt = (int)blockDim.x;
  for (int i0 = (int)threadIdx.x; i0 < total; i0 += 4 * nt) {
    Cx<T> v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int idx = i0 + u * nt;
      const int p = idx / LB, l = idx - p * LB;
      const bool use = idx < total && ok(p, l);
      const Cx<T> x = ld(use ? addr(p, l) : safe);
      v[u] = use ? x : Cx<T>{0, 0};
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int idx = i0 + u * nt;
      if (idx < total) {
        const int p = idx / LB, l = idx - p * LB;
        buf[l * (M + 1) + p] = v[u];
      }
    }
  }
}

// cyclic index of the ghost-inclusive position p = 0..n+1 (node p - 1): M - 1 for p = 0
__device__ __forceinline__ int ghost_src(int p, int M) { return p == 0 ? M - 1 : p - 1; }

// Three uses of the same passes.  MODE 0 (Poisson solve): the source lives on nodes 0..n-1 and
// the result is kept on nodes -1..n.  MODE 1 (transposed solve of the reverse sweep): the
// source lives on nodes -1..n (node -1 at cyclic index M - 1) and the result is kept on nodes
// 0..n-1.  MODE 2 (direct field): source and result on nodes 0..n-1.  All are exact: every
// source-to-output offset lies in [-n, n].
template <int MODE>
__device__ __forceinline__ bool src_nonzero(int p, int n, int M) {
  return MODE != 1 ? p < n : (p <= n || p == M - 1);
}
template <int MODE>
__device__ __forceinline__ int out_count(int n) { return MODE == 0 ? n + 2 : n; }
template <int MODE>
__device__ __forceinline__ int out_src(int q, int M) { return MODE == 0 ? ghost_src(q, M) : q; }
__device__ __forceinline__ int fold(int k, int M) { return k <= M / 2 ? k : M - k; }

// ------------------------------------------------------------------------------ Green spectrum

// Even-real DFT along one axis of the float64 array gd[(k (ny+1) + j)(nx+1) + i] in place:
// line values g_0..g_n are extended to length M = 2n by g_t = g_{M-t}, transformed, and the
// real outputs k = 0..n stored.  Complex line c carries real lines a = 2c (real part) and
// a = 2c + 1 (imaginary part); line a starts at a*sa + b*sb, elements at stride st.
// ODD: the odd extension g_t = -g_{M-t} (g_n = 0, an offset no output node reaches), whose
// transform is i S_k with S real; S is stored (the factor i is applied by the product).  For
// a packed pair Z = A + i B with A = i S_A, B = i S_B: S_A = Im Z, S_B = -Re Z.
template <bool ODD>
__device__ __forceinline__ void green_dft_body(double* __restrict__ gd, FftAxis ax,
                                                         const double2* __restrict__ tw,
                                                         int64_t st, int64_t sa, int64_t sb,
                                                         int na, int LB, int bx, int by, int nbx) {
  extern __shared__ unsigned char smem_raw[];
  Cx<double>* buf = reinterpret_cast<Cx<double>*>(smem_raw);
  const int M = ax.M, n = M / 2;
  const int c0 = bx * LB;  // first complex line of this block
  double* base = gd + (int64_t)by * sb;
  // consecutive threads take consecutive elements of a line where the line is contiguous in
  // memory (st == 1), else consecutive lines (contiguous across lines)
  const bool efast = st == 1;
  for (int idx = threadIdx.x; idx < LB * M; idx += blockDim.x) {
    int p, l;
    if (efast) {
      l = idx / M;
      p = idx - l * M;
    } else {
      p = idx / LB;
      l = idx - p * LB;
    }
    const int t = p <= n ? p : M - p;
    const double sgn = ODD ? (p < n ? 1.0 : (p == n ? 0.0 : -1.0)) : 1.0;
    const int a0 = 2 * (c0 + l), a1 = a0 + 1;
    double re = a0 < na ? base[(int64_t)a0 * sa + (int64_t)t * st] : 0.0;
    double im = a1 < na ? base[(int64_t)a1 * sa + (int64_t)t * st] : 0.0;
    buf[l * (M + 1) + p] = Cx<double>{sgn * re, sgn * im};
  }
  const double2* twl = stage_twiddles(buf, LB, M, tw, M);
  __syncthreads();
  fft_lds<double, -1>(buf, LB, ax, twl, 1);
  for (int idx = threadIdx.x; idx < LB * (n + 1); idx += blockDim.x) {
    int p, l;
    if (efast) {
      l = idx / (n + 1);
      p = idx - l * (n + 1);
    } else {
      p = idx / LB;
      l = idx - p * LB;
    }
    const int a0 = 2 * (c0 + l), a1 = a0 + 1;
    const Cx<double> v = buf[l * (M + 1) + p];
    if (a0 < na) base[(int64_t)a0 * sa + (int64_t)p * st] = ODD ? v.y : v.x;
    if (a1 < na) base[(int64_t)a1 * sa + (int64_t)p * st] = ODD ? -v.x : v.y;
  }
}

__device__ __forceinline__ void green_even_dft_body(double* __restrict__ gd, FftAxis ax,
                                                    const double2* __restrict__ tw, int64_t st,
                                                    int64_t sa, int64_t sb, int na, int LB,
                                                    int bx, int by, int nbx) {
  green_dft_body<false>(gd, ax, tw, st, sa, sb, na, LB, bx, by, nbx);
}

template <bool ODD>
__global__ __launch_bounds__(1024) void k_green_dft(double* __restrict__ gd, FftAxis ax,
                                                    const double2* __restrict__ tw, int64_t st,
                                                    int64_t sa, int64_t sb, int na, int LB) {
  green_dft_body<ODD>(gd, ax, tw, st, sa, sb, na, LB, blockIdx.x, blockIdx.y, gridDim.x);
}

template <typename T>
__device__ __forceinline__ void green_finish_body(const Geom* __restrict__ g,
                                                      const double* __restrict__ gd,
                                                      T* __restrict__ gh, int64_t total,
                                                      double scale, int bx, int by, int nbx) {
  if (g->status) return;
  for (int64_t t = bx * 256ll + threadIdx.x; t < total; t += (int64_t)nbx * 256)
    gh[t] = (T)(gd[t] * scale);
}

template <typename T>
__global__ __launch_bounds__(256) void k_green_finish(const Geom* __restrict__ g,
                                                      const double* __restrict__ gd,
                                                      T* __restrict__ gh, int64_t total,
                                                      double scale) {
  green_finish_body<T>(g, gd, gh, total, scale, blockIdx.x, blockIdx.y, gridDim.x);
}

// ------------------------------------------------------------------------------ solve passes

// Forward real transform of the source rows into the half spectrum W[z][y][0..n_x], z and y
// cyclic.  MODE 0: rows (y < n_y, z < n_z) of the charge src[z][y][x] (length n_x).  MODE 1:
// rows (yy < n_y + 2, zz < n_z + 2) of the ghost-inclusive source src[zz][yy][xx]
// (length n_x + 2, node xx - 1), stored at cyclic rows (ghost_src(zz), ghost_src(yy)).
// Packed z_j = x_{2j} + i x_{2j+1}, j < n_x, complex FFT of length n_x (ax), then
// X_k = E_k + W^k O_k, E_k = (Z_k + conj Z_{n-k})/2, O_k = (Z_k - conj Z_{n-k})/(2i),
// W = exp(-2 pi i / M_x), k = 0..n_x.
template <typename T, int MODE>
__device__ __forceinline__ void r2c_x_body(const Geom* __restrict__ g,
                                                const T* __restrict__ src, Cx<T>* __restrict__ W,
                                                FftAxis ax, const typename TwT<T>::type* __restrict__ tw,
                                                int nx, int ny, int nz, int Kx, int My, int LB, int bx, int by, int nbx) {
  extern __shared__ unsigned char smem_raw[];
  Cx<T>* buf = reinterpret_cast<Cx<T>*>(smem_raw);
  if (g->status) return;
  const int H = ax.M;  // = nx
  const int M = 2 * H;
  const int rows = MODE == 0 ? ny : ny + 2;
  const int len = MODE == 0 ? nx : nx + 2;
  const int y0 = bx * LB, z = by;
  const int nl = min(LB, rows - y0);
  const T* s0 = src + ((int64_t)z * rows + y0) * len;
  // four elements per thread at a time, their loads issued before any is stored and with no
  // branch around a load (out-of-range addresses replaced by the row's start, values by zero)
  const int total = LB * H, nt = (int)blockDim.x;
  for (int i0 = (int)threadIdx.x; i0 < total; i0 += 4 * nt) {
    T vr[4][2];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int idx = i0 + u * nt;
      const int l = idx / H, j = idx - l * H;
      const bool row_ok = idx < total && l < nl;
      const T* row = s0 + (int64_t)(row_ok ? l : 0) * len;
#pragma unroll
      for (int h2 = 0; h2 < 2; ++h2) {
        const int t = 2 * j + h2;  // cyclic position
        int at = -1;               // its element in the source row, if any
        if (MODE == 0) {
          if (t < nx) at = t;
        } else {
          if (t <= nx) at = t + 1;
          else if (t == M - 1) at = 0;
        }
        const bool use = row_ok && at >= 0;
        const T val = row[use ? at : 0];
        vr[u][h2] = use ? val : T(0);
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int idx = i0 + u * nt;
      if (idx < total) {
        const int l = idx / H, j = idx - l * H;
        buf[l * (H + 1) + j] = Cx<T>{vr[u][0], vr[u][1]};
      }
    }
  }
  const auto* twl = stage_twiddles(buf, LB, H, tw, M);
  __syncthreads();
  fft_lds<T, -1>(buf, LB, ax, twl, 2);
  const int cz = MODE == 0 ? z : ghost_src(z, 2 * nz);
  for (int idx = threadIdx.x; idx < LB * (H + 1); idx += blockDim.x) {
    const int l = idx / (H + 1), k = idx - l * (H + 1);
    if (l >= nl) continue;
    const int cy = MODE == 0 ? y0 + l : ghost_src(y0 + l, My);
    const Cx<T> zk = buf[l * (H + 1) + (k % H)];
    const Cx<T> zc = cconj(buf[l * (H + 1) + ((H - k) % H)]);
    const Cx<T> e = {(T)0.5 * (zk.x + zc.x), (T)0.5 * (zk.y + zc.y)};
    const Cx<T> dif = csub(zk, zc);
    const Cx<T> o = {(T)0.5 * dif.y, (T)-0.5 * dif.x};  // dif / (2i)
    const auto w = tw[k];                              // exp(-2 pi i k / M_x)
    W[((int64_t)cz * My + cy) * Kx + k] = cadd(e, cmul(Cx<T>{(T)w.x, (T)w.y}, o));
  }
}

template <typename T, int MODE>
__global__ __launch_bounds__(1024) void k_r2c_x(const Geom* __restrict__ g,
                                                const T* __restrict__ src, Cx<T>* __restrict__ W,
                                                FftAxis ax, const typename TwT<T>::type* __restrict__ tw,
                                                int nx, int ny, int nz, int Kx, int My, int LB) {
  r2c_x_body<T, MODE>(g, src, W, ax, tw, nx, ny, nz, Kx, My, LB, blockIdx.x, blockIdx.y, gridDim.x);
}

// Complex line FFT in place along y (element stride Kx) for lines a = kx (stride 1) on the
// planes b = blockIdx.y.  STAGE 0 (forward): the planes holding source rows -- z < n_z
// (MODE 0) or the cyclic rows of nodes -1..n_z (MODE 1) -- with the source's non-zero inputs
// only, all M outputs stored.  STAGE 1 (inverse): the planes b < out_count(n_z) written by the
// z pass, all M inputs, the out_count(n_y) kept rows stored at positions q from out_src(q).
template <typename T, int DIR, int MODE, int STAGE>
__device__ __forceinline__ void c2c_y_body(const Geom* __restrict__ g, Cx<T>* __restrict__ W,
                                                FftAxis ax,
                                                const typename TwT<T>::type* __restrict__ tw,
                                                int Kx, int ny, int nz, int LB, int bx, int by, int nbx) {
  extern __shared__ unsigned char smem_raw[];
  Cx<T>* buf = reinterpret_cast<Cx<T>*>(smem_raw);
  if (g->status) return;
  const int M = ax.M;
  const int a0 = bx * LB;
  const int nl = min(LB, Kx - a0);
  const int plane = (STAGE == 0 && MODE == 1) ? ghost_src(by, 2 * nz) : (int)by;
  Cx<T>* base = W + (int64_t)plane * M * Kx + a0;
  load_lines<T>(
      buf, LB, M, base, [&](int p, int l) { return base + (int64_t)p * Kx + l; },
      [&](int p, int l) { return l < nl && (STAGE == 1 || src_nonzero<MODE>(p, ny, M)); });
  const auto* twl = stage_twiddles(buf, LB, M, tw, M);
  __syncthreads();
  fft_lds<T, DIR>(buf, LB, ax, twl, 1);
  const int nout = STAGE == 0 ? M : out_count<MODE>(ny);
  for (int idx = threadIdx.x; idx < LB * nout; idx += blockDim.x) {
    const int q = idx / LB, l = idx - q * LB;
    if (l < nl)
      base[(int64_t)q * Kx + l] = buf[l * (M + 1) + (STAGE == 0 ? q : out_src<MODE>(q, M))];
  }
}

template <typename T, int DIR, int MODE, int STAGE>
__global__ __launch_bounds__(1024) void k_c2c_y(const Geom* __restrict__ g, Cx<T>* __restrict__ W,
                                                FftAxis ax,
                                                const typename TwT<T>::type* __restrict__ tw,
                                                int Kx, int ny, int nz, int LB) {
  c2c_y_body<T, DIR, MODE, STAGE>(g, W, ax, tw, Kx, ny, nz, LB, blockIdx.x, blockIdx.y, gridDim.x);
}

// Along z (element stride My Kx) for lines a = kx, b = ky: forward FFT of the source's
// non-zero inputs, product with Ghat(fold kz, fold ky, kx) (gh[(fz (ny+1) + fy)(nx+1) + kx]),
// inverse FFT, and the out_count(n_z) kept rows written back in place.
// IMAG: the kernel spectrum is i gh (an odd field kernel, see green_dft_body), odd along axis
// `odd`: its spectrum is odd there too, so the folded value changes sign for k_y > n_y
// (odd = 1) or k_z > n_z (odd = 2); along x only k_x <= n_x is stored, no fold.  W2: where the
// kept rows go (W itself for the potential).
template <typename T, int MODE, bool IMAG = false>
__device__ __forceinline__ void zconv_body(const Geom* __restrict__ g, Cx<T>* W,
                                                const T* __restrict__ gh, FftAxis ax,
                                                const typename TwT<T>::type* __restrict__ tw,
                                                int Kx, int My, int ny, int nz, int LB, int bx, int by, int nbx,
                                                Cx<T>* W2 = nullptr, int odd = -1) {
  extern __shared__ unsigned char smem_raw[];
  Cx<T>* buf = reinterpret_cast<Cx<T>*>(smem_raw);
  if (g->status) return;
  const int M = ax.M;
  const int a0 = bx * LB, ky = by;
  const int nl = min(LB, Kx - a0);
  const int64_t sz = (int64_t)My * Kx;
  Cx<T>* base = W + (int64_t)ky * Kx + a0;
  Cx<T>* obase = (W2 ? W2 : W) + (int64_t)ky * Kx + a0;
  load_lines<T>(
      buf, LB, M, base, [&](int p, int l) { return base + (int64_t)p * sz + l; },
      [&](int p, int l) { return l < nl && src_nonzero<MODE>(p, nz, M); });
  const auto* twl = stage_twiddles(buf, LB, M, tw, M);
  const int fy = fold(ky, My);
  const T* grow = gh + (int64_t)fy * Kx + a0;
  const int64_t gplane = (int64_t)(ny + 1) * Kx;
  const bool flip_y = IMAG && odd == 1 && ky > ny;
  const int total = LB * M, nt = (int)blockDim.x;
  __syncthreads();
  fft_lds<T, -1>(buf, LB, ax, twl, 1);
  // the kernel spectrum of the thread's first 4 elements (all of them with the launches'
  // shapes, LB M <= 4 blockDim.x), loaded together without a branch around a load (loading it
  // before the transform would hold 8 more registers through it and halve the resident blocks)
  T gs[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int idx = (int)threadIdx.x + u * nt;
    const int p = idx / LB, l = idx - p * LB;
    const bool use = idx < total && l < nl;
    gs[u] = grow[use ? (int64_t)fold(p, M) * gplane + l : 0];
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int idx = (int)threadIdx.x + u * nt;
    const int p = idx / LB, l = idx - p * LB;
    if (idx < total && l < nl) {
      T s = gs[u];
      if (IMAG && (flip_y || (odd == 2 && p > nz))) s = -s;
      Cx<T> v = buf[l * (M + 1) + p];
      buf[l * (M + 1) + p] = IMAG ? Cx<T>{-v.y * s, v.x * s} : Cx<T>{v.x * s, v.y * s};
    }
  }
  // elements past 4 blockDim.x (none with the launches' shapes) load their spectrum here
  for (int idx = (int)threadIdx.x + 4 * nt; idx < total; idx += nt) {
    const int p = idx / LB, l = idx - p * LB;
    if (l < nl) {
      T s = grow[(int64_t)fold(p, M) * gplane + l];
      if (IMAG && (flip_y || (odd == 2 && p > nz))) s = -s;
      Cx<T> v = buf[l * (M + 1) + p];
      buf[l * (M + 1) + p] = IMAG ? Cx<T>{-v.y * s, v.x * s} : Cx<T>{v.x * s, v.y * s};
    }
  }
  __syncthreads();
  fft_lds<T, +1>(buf, LB, ax, twl, 1);
  for (int idx = threadIdx.x; idx < LB * out_count<MODE>(nz); idx += blockDim.x) {
    const int q = idx / LB, l = idx - q * LB;
    if (l < nl) obase[(int64_t)q * sz + l] = buf[l * (M + 1) + out_src<MODE>(q, M)];
  }
}

template <typename T, int MODE>
__global__ __launch_bounds__(1024) void k_zconv(const Geom* __restrict__ g, Cx<T>* __restrict__ W,
                                                const T* __restrict__ gh, FftAxis ax,
                                                const typename TwT<T>::type* __restrict__ tw,
                                                int Kx, int My, int ny, int nz, int LB) {
  zconv_body<T, MODE>(g, W, gh, ax, tw, Kx, My, ny, nz, LB, blockIdx.x, blockIdx.y, gridDim.x);
}

// direct field: forward z FFT of W (kept intact for the next component), product with i gh,
// inverse z FFT, the n_z node rows into W2 [n_z][2 n_y][n_x + 1]
template <typename T>
__global__ __launch_bounds__(1024) void k_zconv_field(const Geom* __restrict__ g,
                                                      Cx<T>* __restrict__ W,
                                                      const T* __restrict__ gh, FftAxis ax,
                                                      const typename TwT<T>::type* __restrict__ tw,
                                                      int Kx, int My, int ny, int nz, int LB,
                                                      Cx<T>* __restrict__ W2, int odd) {
  zconv_body<T, 2, true>(g, W, gh, ax, tw, Kx, My, ny, nz, LB, blockIdx.x, blockIdx.y, gridDim.x,
                         W2, odd);
}

// Inverse real transform of the kept rows (yy < out_count(n_y), zz < out_count(n_z)) of W,
// writing the result on the kept x-nodes (MODE 0: -1..n_x into phi[(nz+2)][(ny+2)][(nx+2)];
// MODE 1: 0..n_x-1 into an [nz][ny][nx] array): Z_k = (X_k + conj X_{n-k}) + i exp(+2 pi i k/M_x)(X_k - conj X_{n-k}),
// k < n = n_x, inverse complex FFT of length n_x, x_{2j} = Re z_j, x_{2j+1} = Im z_j.
template <typename T, int MODE>
__device__ __forceinline__ void c2r_x_body(const Geom* __restrict__ g,
                                                const Cx<T>* __restrict__ W, T* __restrict__ phi,
                                                FftAxis ax,
                                                const typename TwT<T>::type* __restrict__ tw,
                                                int nx, int ny, int Kx, int My, int LB, int bx, int by, int nbx) {
  extern __shared__ unsigned char smem_raw[];
  Cx<T>* buf = reinterpret_cast<Cx<T>*>(smem_raw);
  if (g->status) return;
  const int H = ax.M;  // = nx
  const int M = 2 * H;
  const int py = out_count<MODE>(ny);
  const int r0 = bx * LB, zz = by;
  const int nl = min(LB, py - r0);
  const Cx<T>* src = W + ((int64_t)zz * My + r0) * Kx;
  // four elements per thread at a time, their loads issued before any is used and with no
  // branch around a load (rows past the block's last read as row 0, their values not used)
  const int total = LB * H, nt = (int)blockDim.x;
  for (int i0 = (int)threadIdx.x; i0 < total; i0 += 4 * nt) {
    Cx<T> xk[4], xh[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int idx = i0 + u * nt;
      const int l = idx / H, k = idx - l * H;
      const bool ok = idx < total && l < nl;
      const Cx<T>* row = src + (int64_t)(ok ? l : 0) * Kx;
      const int kk = ok ? k : 0;
      xk[u] = ld(row + kk);
      xh[u] = ld(row + (H - kk));
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int idx = i0 + u * nt;
      if (idx < total) {
        const int l = idx / H, k = idx - l * H;
        const auto w = tw[k];
        Cx<T> v = {0, 0};
        if (l < nl) {
          const Cx<T> xc = cconj(xh[u]);
          const Cx<T> winv = {(T)w.x, (T)-w.y};  // exp(+2 pi i k / M_x)
          const Cx<T> d = cmul(winv, csub(xk[u], xc));
          v = cadd(cadd(xk[u], xc), Cx<T>{-d.y, d.x});  // + i d
        }
        buf[l * (H + 1) + k] = v;
      }
    }
  }
  const auto* twl = stage_twiddles(buf, LB, H, tw, M);
  __syncthreads();
  fft_lds<T, +1>(buf, LB, ax, twl, 2);
  const int px = out_count<MODE>(nx);
  T* dst = phi + ((int64_t)zz * py + r0) * px;
  for (int idx = threadIdx.x; idx < LB * px; idx += blockDim.x) {
    const int l = idx / px, q = idx - l * px;
    if (l < nl) {
      const int t = out_src<MODE>(q, M);
      const Cx<T> zj = buf[l * (H + 1) + (t >> 1)];
      dst[(int64_t)l * px + q] = (t & 1) ? zj.y : zj.x;
    }
  }
}

template <typename T, int MODE>
__global__ __launch_bounds__(1024) void k_c2r_x(const Geom* __restrict__ g,
                                                const Cx<T>* __restrict__ W, T* __restrict__ phi,
                                                FftAxis ax,
                                                const typename TwT<T>::type* __restrict__ tw,
                                                int nx, int ny, int Kx, int My, int LB) {
  c2r_x_body<T, MODE>(g, W, phi, ax, tw, nx, ny, Kx, My, LB, blockIdx.x, blockIdx.y, gridDim.x);
}

// E'[c][k][j][i] = -(phi(n + e_c) - phi(n - e_c)) / (2 h_c), rest-frame spacings
template <typename T>
__device__ __forceinline__ void grad_body(const Geom* __restrict__ g, const T* __restrict__ phi,
                                              T* __restrict__ E, int nx, int ny, int nz, int bx, int by, int nbx) {
  if (g->status) return;
  const int px = nx + 2, py = ny + 2;
  const int64_t total = (int64_t)nx * ny * nz;
  const T cx = (T)(1.0 / (2.0 * g->h_rest[0]));
  const T cy = (T)(1.0 / (2.0 * g->h_rest[1]));
  const T cz = (T)(1.0 / (2.0 * g->h_rest[2]));
  const int64_t sy = px, sz = (int64_t)px * py;
  for (int64_t t = bx * 256ll + threadIdx.x; t < total; t += (int64_t)nbx * 256) {
    int i = (int)(t % nx), j = (int)((t / nx) % ny), k = (int)(t / ((int64_t)nx * ny));
    int64_t c = (int64_t)(k + 1) * sz + (int64_t)(j + 1) * sy + (i + 1);
    E[t] = -(phi[c + 1] - phi[c - 1]) * cx;
    E[total + t] = -(phi[c + sy] - phi[c - sy]) * cy;
    E[2 * total + t] = -(phi[c + sz] - phi[c - sz]) * cz;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_grad(const Geom* __restrict__ g, const T* __restrict__ phi,
                                              T* __restrict__ E, int nx, int ny, int nz) {
  grad_body<T>(g, phi, E, nx, ny, nz, blockIdx.x, blockIdx.y, gridDim.x);
}


// ------------------------------------------------------------------------ batched wrappers
// beam = blockIdx.z; lines per workgroup as in shape_for, per beam; blocks beyond a beam's
// extent exit.

template <typename T>
__device__ __forceinline__ const typename TwT<T>::type* tw_of(const FftPlan& p, int a);
template <>
__device__ __forceinline__ const double2* tw_of<double>(const FftPlan& p, int a) { return p.tw[a]; }
template <>
__device__ __forceinline__ const float2* tw_of<float>(const FftPlan& p, int a) { return p.twf[a]; }

__device__ __forceinline__ int lines_per_block(int L, int lines) {
  int lb = kLdsElems / (L + 1);
  if (lb < 1) lb = 1;
  return lb > lines ? lines : lb;
}

__global__ __launch_bounds__(1024) void k_green_even_dft_batch(const BeamDev* __restrict__ beams,
                                                               int axis) {
  const BeamDev& d = beams[blockIdx.z];
  if (d.geom->status) return;
  const int ex = d.c.nx + 1, ey = d.c.ny + 1, ez = d.c.nz + 1;
  int64_t st, sa, sb;
  int na, nplanes;
  if (axis == 0) {
    st = 1; sa = ex; sb = (int64_t)ex * ey; na = ey; nplanes = ez;
  } else if (axis == 1) {
    st = ex; sa = 1; sb = (int64_t)ex * ey; na = ex; nplanes = ez;
  } else {
    st = (int64_t)ex * ey; sa = 1; sb = 0; na = ex * ey; nplanes = 1;
  }
  const int ncx = (na + 1) / 2;
  const int LB = lines_per_block(d.plan.full[axis].M, ncx);
  if ((int)blockIdx.x >= (ncx + LB - 1) / LB || (int)blockIdx.y >= nplanes) return;
  green_even_dft_body(d.Gd, d.plan.full[axis], d.plan.tw[axis], st, sa, sb, na, LB, blockIdx.x,
                      blockIdx.y, gridDim.x);
}

template <typename T>
__global__ __launch_bounds__(256) void k_green_finish_batch(const BeamDev* __restrict__ beams) {
  const BeamDev& d = beams[blockIdx.y];
  const int64_t total = (int64_t)(d.c.nx + 1) * (d.c.ny + 1) * (d.c.nz + 1);
  const double scale = 1.0 / (4.0 * 3.14159265358979323846 * 8.8541878128e-12 *
                              (8.0 * d.c.nx * d.c.ny * d.c.nz));
  green_finish_body<T>(d.geom, d.Gd, (T*)d.Gh, total, scale, blockIdx.x, 0, gridDim.x);
}

template <typename T>
__global__ __launch_bounds__(1024) void k_r2c_x_batch(const BeamDev* __restrict__ beams) {
  const BeamDev& d = beams[blockIdx.z];
  const int nx = d.c.nx, ny = d.c.ny, nz = d.c.nz;
  const int LB = lines_per_block(d.plan.half_x.M, ny);
  if ((int)blockIdx.x >= (ny + LB - 1) / LB || (int)blockIdx.y >= nz) return;
  r2c_x_body<T, 0>(d.geom, (const T*)d.rho, (Cx<T>*)d.W, d.plan.half_x, tw_of<T>(d.plan, 0), nx,
                   ny, nz, nx + 1, 2 * ny, LB, blockIdx.x, blockIdx.y, gridDim.x);
}

template <typename T, int DIR, int STAGE>
__global__ __launch_bounds__(1024) void k_c2c_y_batch(const BeamDev* __restrict__ beams) {
  const BeamDev& d = beams[blockIdx.z];
  const int Kx = d.c.nx + 1, ny = d.c.ny, nz = d.c.nz;
  const int LB = lines_per_block(d.plan.full[1].M, Kx);
  const int planes = STAGE == 0 ? nz : nz + 2;
  if ((int)blockIdx.x >= (Kx + LB - 1) / LB || (int)blockIdx.y >= planes) return;
  c2c_y_body<T, DIR, 0, STAGE>(d.geom, (Cx<T>*)d.W, d.plan.full[1], tw_of<T>(d.plan, 1), Kx, ny,
                               nz, LB, blockIdx.x, blockIdx.y, gridDim.x);
}

template <typename T>
__global__ __launch_bounds__(1024) void k_zconv_batch(const BeamDev* __restrict__ beams) {
  const BeamDev& d = beams[blockIdx.z];
  const int Kx = d.c.nx + 1, My = 2 * d.c.ny;
  const int LB = lines_per_block(d.plan.full[2].M, Kx);
  if ((int)blockIdx.x >= (Kx + LB - 1) / LB || (int)blockIdx.y >= My) return;
  zconv_body<T, 0>(d.geom, (Cx<T>*)d.W, (const T*)d.Gh, d.plan.full[2], tw_of<T>(d.plan, 2), Kx,
                   My, d.c.ny, d.c.nz, LB, blockIdx.x, blockIdx.y, gridDim.x);
}

template <typename T>
__global__ __launch_bounds__(1024) void k_c2r_x_batch(const BeamDev* __restrict__ beams) {
  const BeamDev& d = beams[blockIdx.z];
  const int nx = d.c.nx, ny = d.c.ny, nz = d.c.nz;
  const int LB = lines_per_block(d.plan.half_x.M, ny + 2);
  if ((int)blockIdx.x >= (ny + 2 + LB - 1) / LB || (int)blockIdx.y >= nz + 2) return;
  c2r_x_body<T, 0>(d.geom, (const Cx<T>*)d.W, (T*)d.phi, d.plan.half_x, tw_of<T>(d.plan, 0), nx,
                   ny, nx + 1, 2 * ny, LB, blockIdx.x, blockIdx.y, gridDim.x);
}

template <typename T>
__global__ __launch_bounds__(256) void k_grad_batch(const BeamDev* __restrict__ beams) {
  const BeamDev& d = beams[blockIdx.y];
  grad_body<T>(d.geom, (const T*)d.phi, (T*)d.E, d.c.nx, d.c.ny, d.c.nz, blockIdx.x, 0,
               gridDim.x);
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
  int lb = kLdsElems / (L + 1);
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

namespace {
// The three even/odd DFT passes of one octant kernel gd (odd_axis: -1 for an even kernel) and
// the scaled conversion into gh.
template <typename T>
hipError_t kernel_spectrum(const Geom* g, const FftPlan& p, int nx, int ny, int nz, double* gd,
                           T* gh, int odd_axis, hipStream_t s) {
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
    size_t lds = (size_t)LB * (p.full[a].M + 1) * sizeof(Cx<double>) +
                 (size_t)p.full[a].M * sizeof(double2);
    if (a == odd_axis)
      hipLaunchKernelGGL(k_green_dft<true>, grid, dim3(NT), lds, s, gd, p.full[a], p.tw[a],
                         cfg[a][0], cfg[a][1], cfg[a][2], na, LB);
    else
      hipLaunchKernelGGL(k_green_dft<false>, grid, dim3(NT), lds, s, gd, p.full[a], p.tw[a],
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
}  // namespace

template <typename T>
hipError_t launch_green_field_spectrum(const Geom* g, const FftPlan& p, int nx, int ny, int nz,
                                       double2* hcorners, double* gd3, T* gh3, hipStream_t s) {
  PIC_TRY(launch_igf_field(g, nx, ny, nz, hcorners, gd3, s));
  const int64_t total = (int64_t)(nx + 1) * (ny + 1) * (nz + 1);
  for (int a = 0; a < 3; ++a)
    PIC_TRY(kernel_spectrum<T>(g, p, nx, ny, nz, gd3 + a * total, gh3 + a * total, a, s));
  return hipSuccess;
}

template <typename T>
hipError_t launch_green_dh_spectra(const Geom* g, const FftPlan& p, int nx, int ny, int nz,
                                   bool field, double2* dc, double* gd, T* gh, hipStream_t s) {
  PIC_TRY(launch_igf_dh(g, nx, ny, nz, field, dc, gd, s));
  const int64_t total = (int64_t)(nx + 1) * (ny + 1) * (nz + 1);
  if (!field) {
    for (int b = 0; b < 3; ++b)
      PIC_TRY(kernel_spectrum<T>(g, p, nx, ny, nz, gd + b * total, gh + b * total, -1, s));
    return hipSuccess;
  }
  // kernel (a, b) = f = 3 a + b in gd; its spectrum at 3 b + a, so that the three of one b
  // are consecutive, as the transposed field solve reads them
  for (int f = 0; f < 9; ++f)
    PIC_TRY(kernel_spectrum<T>(g, p, nx, ny, nz, gd + f * total,
                               gh + (3 * (f % 3) + f / 3) * total, f / 3, s));
  return hipSuccess;
}

template <typename T>
hipError_t launch_green_spectrum(const Geom* g, const FftPlan& p, int nx, int ny, int nz,
                                 double2* corners, double* gd, T* gh, hipStream_t s) {
  PIC_TRY(launch_igf_corners(g, nx, ny, nz, corners, s));
  PIC_TRY(launch_igf_cells(g, nx, ny, nz, corners, gd, s));
  return kernel_spectrum<T>(g, p, nx, ny, nz, gd, gh, -1, s);
}


namespace {

// MODE 0: phi (nodes -1..n) from rho (nodes 0..n-1); MODE 1: chi (nodes 0..n-1) from a source
// on nodes -1..n.  src/dst layouts as in k_r2c_x and k_c2r_x.
template <typename T, int MODE>
hipError_t run_passes(const Geom* g, const FftPlan& p, int nx, int ny, int nz, const T* src,
                      Cx<T>* W, const T* gh, T* dst, hipStream_t s) {
  const int My = 2 * ny, Kx = nx + 1;
  const int rows_y = MODE == 0 ? ny : ny + 2, rows_z = MODE == 0 ? nz : nz + 2;
  const int out_y = MODE == 0 ? ny + 2 : ny, out_z = MODE == 0 ? nz + 2 : nz;
  int LB, NT;
  size_t lds;
  shape_for(p.half_x.M, rows_y, &LB, &NT);
  lds = (size_t)LB * (p.half_x.M + 1) * sizeof(Cx<T>) +
        (size_t)p.full[0].M * sizeof(typename TwT<T>::type);
  hipLaunchKernelGGL((k_r2c_x<T, MODE>), dim3((rows_y + LB - 1) / LB, rows_z), dim3(NT), lds, s,
                     g, src, W, p.half_x, table<T>(p, 0), nx, ny, nz, Kx, My, LB);
  PIC_TRY(hipGetLastError());
  shape_for(p.full[1].M, Kx, &LB, &NT);
  lds = (size_t)LB * (p.full[1].M + 1) * sizeof(Cx<T>) +
        (size_t)p.full[1].M * sizeof(typename TwT<T>::type);
  hipLaunchKernelGGL((k_c2c_y<T, -1, MODE, 0>), dim3((Kx + LB - 1) / LB, rows_z), dim3(NT), lds,
                     s, g, W, p.full[1], table<T>(p, 1), Kx, ny, nz, LB);
  PIC_TRY(hipGetLastError());
  shape_for(p.full[2].M, Kx, &LB, &NT);
  lds = (size_t)LB * (p.full[2].M + 1) * sizeof(Cx<T>) +
        (size_t)p.full[2].M * sizeof(typename TwT<T>::type);
  hipLaunchKernelGGL((k_zconv<T, MODE>), dim3((Kx + LB - 1) / LB, My), dim3(NT), lds, s, g, W,
                     gh, p.full[2], table<T>(p, 2), Kx, My, ny, nz, LB);
  PIC_TRY(hipGetLastError());
  shape_for(p.full[1].M, Kx, &LB, &NT);
  lds = (size_t)LB * (p.full[1].M + 1) * sizeof(Cx<T>) +
        (size_t)p.full[1].M * sizeof(typename TwT<T>::type);
  hipLaunchKernelGGL((k_c2c_y<T, +1, MODE, 1>), dim3((Kx + LB - 1) / LB, out_z), dim3(NT), lds,
                     s, g, W, p.full[1], table<T>(p, 1), Kx, ny, nz, LB);
  PIC_TRY(hipGetLastError());
  shape_for(p.half_x.M, out_y, &LB, &NT);
  lds = (size_t)LB * (p.half_x.M + 1) * sizeof(Cx<T>) +
        (size_t)p.full[0].M * sizeof(typename TwT<T>::type);
  hipLaunchKernelGGL((k_c2r_x<T, MODE>), dim3((out_y + LB - 1) / LB, out_z), dim3(NT), lds, s, g,
                     W, dst, p.half_x, table<T>(p, 0), nx, ny, Kx, My, LB);
  return hipGetLastError();
}

}  // namespace

template <typename T>
hipError_t launch_solve(const Geom* g, const FftPlan& p, int nx, int ny, int nz, const T* rho,
                        void* Wv, const T* gh, T* phi, T* E, hipStream_t s) {
  PIC_TRY((run_passes<T, 0>(g, p, nx, ny, nz, rho, (Cx<T>*)Wv, gh, phi, s)));
  const int64_t ng = (int64_t)nx * ny * nz;
  hipLaunchKernelGGL((k_grad<T>), dim3(grid_for(ng)), dim3(256), 0, s, g, phi, E, nx, ny, nz);
  return hipGetLastError();
}

// Direct field: forward x and y passes of rho into W, then per component the z pass with the
// product by i Ghat_a into W2 and the inverse y and x passes into E_a (nodes 0..n-1).
template <typename T>
hipError_t launch_solve_field(const Geom* g, const FftPlan& p, int nx, int ny, int nz,
                              const T* rho, void* Wv, void* W2v, const T* gh3, T* E,
                              hipStream_t s) {
  Cx<T>* W = (Cx<T>*)Wv;
  Cx<T>* W2 = (Cx<T>*)W2v;
  const int My = 2 * ny, Kx = nx + 1;
  const int64_t ng = (int64_t)nx * ny * nz, gtot = (int64_t)(nx + 1) * (ny + 1) * (nz + 1);
  int LB, NT;
  size_t lds;
  shape_for(p.half_x.M, ny, &LB, &NT);
  lds = (size_t)LB * (p.half_x.M + 1) * sizeof(Cx<T>) +
        (size_t)p.full[0].M * sizeof(typename TwT<T>::type);
  hipLaunchKernelGGL((k_r2c_x<T, 0>), dim3((ny + LB - 1) / LB, nz), dim3(NT), lds, s, g, rho, W,
                     p.half_x, table<T>(p, 0), nx, ny, nz, Kx, My, LB);
  PIC_TRY(hipGetLastError());
  shape_for(p.full[1].M, Kx, &LB, &NT);
  lds = (size_t)LB * (p.full[1].M + 1) * sizeof(Cx<T>) +
        (size_t)p.full[1].M * sizeof(typename TwT<T>::type);
  hipLaunchKernelGGL((k_c2c_y<T, -1, 0, 0>), dim3((Kx + LB - 1) / LB, nz), dim3(NT), lds, s, g,
                     W, p.full[1], table<T>(p, 1), Kx, ny, nz, LB);
  PIC_TRY(hipGetLastError());
  for (int a = 0; a < 3; ++a) {
    shape_for(p.full[2].M, Kx, &LB, &NT);
    lds = (size_t)LB * (p.full[2].M + 1) * sizeof(Cx<T>) +
          (size_t)p.full[2].M * sizeof(typename TwT<T>::type);
    hipLaunchKernelGGL((k_zconv_field<T>), dim3((Kx + LB - 1) / LB, My), dim3(NT), lds, s, g, W,
                       gh3 + a * gtot, p.full[2], table<T>(p, 2), Kx, My, ny, nz, LB, W2, a);
    PIC_TRY(hipGetLastError());
    shape_for(p.full[1].M, Kx, &LB, &NT);
    lds = (size_t)LB * (p.full[1].M + 1) * sizeof(Cx<T>) +
          (size_t)p.full[1].M * sizeof(typename TwT<T>::type);
    hipLaunchKernelGGL((k_c2c_y<T, +1, 2, 1>), dim3((Kx + LB - 1) / LB, nz), dim3(NT), lds, s, g,
                       W2, p.full[1], table<T>(p, 1), Kx, ny, nz, LB);
    PIC_TRY(hipGetLastError());
    shape_for(p.half_x.M, ny, &LB, &NT);
    lds = (size_t)LB * (p.half_x.M + 1) * sizeof(Cx<T>) +
          (size_t)p.full[0].M * sizeof(typename TwT<T>::type);
    hipLaunchKernelGGL((k_c2r_x<T, 2>), dim3((ny + LB - 1) / LB, nz), dim3(NT), lds, s, g, W2,
                       E + a * ng, p.half_x, table<T>(p, 0), nx, ny, Kx, My, LB);
    PIC_TRY(hipGetLastError());
  }
  return hipSuccess;
}

namespace {
// chi = -(t_0 + t_1 + t_2) over the nodes
template <typename T>
__global__ __launch_bounds__(256) void k_neg_sum3(const Geom* __restrict__ g,
                                                  const T* __restrict__ t, int64_t ng,
                                                  T* __restrict__ chi) {
  if (g->status) return;
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < ng; i += (int64_t)gridDim.x * 256)
    chi[i] = -(t[i] + t[ng + i] + t[2 * ng + i]);
}
}  // namespace

// Transpose of launch_solve_field: chi = -sum_a (Kbar_a * e_a) / (4 pi eps0), each a full
// zero-padded convolution (forward x and y passes of e_a, the z pass with i Khat_a, the inverse
// y and x passes onto nodes 0..n-1) into tmp (3 nx ny nz), then the signed sum.
template <typename T>
hipError_t launch_solve_field_T(const Geom* g, const FftPlan& p, int nx, int ny, int nz,
                                const T* e, void* Wv, void* W2v, const T* gh3, T* tmp, T* chi,
                                hipStream_t s) {
  Cx<T>* W = (Cx<T>*)Wv;
  Cx<T>* W2 = (Cx<T>*)W2v;
  const int My = 2 * ny, Kx = nx + 1;
  const int64_t ng = (int64_t)nx * ny * nz, gtot = (int64_t)(nx + 1) * (ny + 1) * (nz + 1);
  for (int a = 0; a < 3; ++a) {
    int LB, NT;
    size_t lds;
    shape_for(p.half_x.M, ny, &LB, &NT);
    lds = (size_t)LB * (p.half_x.M + 1) * sizeof(Cx<T>) +
          (size_t)p.full[0].M * sizeof(typename TwT<T>::type);
    hipLaunchKernelGGL((k_r2c_x<T, 0>), dim3((ny + LB - 1) / LB, nz), dim3(NT), lds, s, g,
                       e + a * ng, W, p.half_x, table<T>(p, 0), nx, ny, nz, Kx, My, LB);
    PIC_TRY(hipGetLastError());
    shape_for(p.full[1].M, Kx, &LB, &NT);
    lds = (size_t)LB * (p.full[1].M + 1) * sizeof(Cx<T>) +
          (size_t)p.full[1].M * sizeof(typename TwT<T>::type);
    hipLaunchKernelGGL((k_c2c_y<T, -1, 0, 0>), dim3((Kx + LB - 1) / LB, nz), dim3(NT), lds, s, g,
                       W, p.full[1], table<T>(p, 1), Kx, ny, nz, LB);
    PIC_TRY(hipGetLastError());
    shape_for(p.full[2].M, Kx, &LB, &NT);
    lds = (size_t)LB * (p.full[2].M + 1) * sizeof(Cx<T>) +
          (size_t)p.full[2].M * sizeof(typename TwT<T>::type);
    hipLaunchKernelGGL((k_zconv_field<T>), dim3((Kx + LB - 1) / LB, My), dim3(NT), lds, s, g, W,
                       gh3 + a * gtot, p.full[2], table<T>(p, 2), Kx, My, ny, nz, LB, W2, a);
    PIC_TRY(hipGetLastError());
    shape_for(p.full[1].M, Kx, &LB, &NT);
    lds = (size_t)LB * (p.full[1].M + 1) * sizeof(Cx<T>) +
          (size_t)p.full[1].M * sizeof(typename TwT<T>::type);
    hipLaunchKernelGGL((k_c2c_y<T, +1, 2, 1>), dim3((Kx + LB - 1) / LB, nz), dim3(NT), lds, s, g,
                       W2, p.full[1], table<T>(p, 1), Kx, ny, nz, LB);
    PIC_TRY(hipGetLastError());
    shape_for(p.half_x.M, ny, &LB, &NT);
    lds = (size_t)LB * (p.half_x.M + 1) * sizeof(Cx<T>) +
          (size_t)p.full[0].M * sizeof(typename TwT<T>::type);
    hipLaunchKernelGGL((k_c2r_x<T, 2>), dim3((ny + LB - 1) / LB, nz), dim3(NT), lds, s, g, W2,
                       tmp + a * ng, p.half_x, table<T>(p, 0), nx, ny, Kx, My, LB);
    PIC_TRY(hipGetLastError());
  }
  int64_t nbk = (ng + 255) / 256;
  if (nbk > 16384) nbk = 16384;
  hipLaunchKernelGGL((k_neg_sum3<T>), dim3((unsigned)nbk), dim3(256), 0, s, g, tmp, ng, chi);
  return hipGetLastError();
}

template hipError_t launch_solve_field_T<double>(const Geom*, const FftPlan&, int, int, int,
                                                 const double*, void*, void*, const double*,
                                                 double*, double*, hipStream_t);
template hipError_t launch_solve_field_T<float>(const Geom*, const FftPlan&, int, int, int,
                                                const float*, void*, void*, const float*,
                                                float*, float*, hipStream_t);

template hipError_t launch_solve_field<double>(const Geom*, const FftPlan&, int, int, int,
                                               const double*, void*, void*, const double*,
                                               double*, hipStream_t);
template hipError_t launch_solve_field<float>(const Geom*, const FftPlan&, int, int, int,
                                              const float*, void*, void*, const float*, float*,
                                              hipStream_t);
template hipError_t launch_green_field_spectrum<double>(const Geom*, const FftPlan&, int, int,
                                                        int, double2*, double*, double*,
                                                        hipStream_t);
template hipError_t launch_green_field_spectrum<float>(const Geom*, const FftPlan&, int, int, int,
                                                       double2*, double*, float*, hipStream_t);

template <typename T>
hipError_t launch_solve_ghost_source(const Geom* g, const FftPlan& p, int nx, int ny, int nz,
                                     const T* psi, void* Wv, const T* gh, T* chi, hipStream_t s) {
  return run_passes<T, 1>(g, p, nx, ny, nz, psi, (Cx<T>*)Wv, gh, chi, s);
}

template hipError_t launch_solve_ghost_source<double>(const Geom*, const FftPlan&, int, int, int,
                                                      const double*, void*, const double*,
                                                      double*, hipStream_t);
template hipError_t launch_solve_ghost_source<float>(const Geom*, const FftPlan&, int, int, int,
                                                     const float*, void*, const float*, float*,
                                                     hipStream_t);
// ------------------------------------------------------------------------ batched launches

namespace {
int ceil_div(int a, int b) { return (a + b - 1) / b; }
int lpb(int L, int lines) {
  int lb = kLdsElems / (L + 1);
  if (lb < 1) lb = 1;
  return lb > lines ? lines : lb;
}
}  // namespace

template <typename T>
hipError_t launch_batch_green(const BeamDev* beams, int nb, const BatchDims& bd, hipStream_t s) {
  PIC_TRY(launch_batch_igf(beams, nb, bd.max_nx, bd.max_ny, bd.max_nz, s));
  const int ex = bd.max_nx + 1, ey = bd.max_ny + 1, ez = bd.max_nz + 1;
  // grid extents over the beams: the largest grid needs the most blocks along every axis
  const int M[3] = {2 * bd.max_nx, 2 * bd.max_ny, 2 * bd.max_nz};
  const int na[3] = {ey, ex, ex * ey}, npl[3] = {ez, ez, 1};
  for (int a = 0; a < 3; ++a) {
    // smaller beams have shorter lines and so at least as many lines per block: the largest
    // beam bounds the block count
    const int ncx = (na[a] + 1) / 2;
    const int gx = ceil_div(ncx, lpb(M[a], ncx));
    hipLaunchKernelGGL(k_green_even_dft_batch, dim3(gx, npl[a], nb), dim3(1024),
                       (size_t)kLdsElems * sizeof(Cx<double>) + 512 * sizeof(double2), s, beams,
                       a);
    PIC_TRY(hipGetLastError());
  }
  const int64_t total = (int64_t)ex * ey * ez;
  hipLaunchKernelGGL((k_green_finish_batch<T>), dim3(grid_for(total), nb), dim3(256), 0, s, beams);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_batch_solve(const BeamDev* beams, int nb, const BatchDims& bd, hipStream_t s) {
  const int nx = bd.max_nx, ny = bd.max_ny, nz = bd.max_nz;
  const int Kx = nx + 1, My = 2 * ny;
  // lines plus a twiddle table of at most 512 entries (2 n <= 512)
  const size_t lds = (size_t)kLdsElems * sizeof(Cx<T>) + 512 * sizeof(typename TwT<T>::type);
  hipLaunchKernelGGL((k_r2c_x_batch<T>), dim3(ceil_div(ny, lpb(nx, ny)), nz, nb), dim3(1024), lds,
                     s, beams);
  PIC_TRY(hipGetLastError());
  hipLaunchKernelGGL((k_c2c_y_batch<T, -1, 0>), dim3(ceil_div(Kx, lpb(My, Kx)), nz, nb),
                     dim3(1024), lds, s, beams);
  PIC_TRY(hipGetLastError());
  hipLaunchKernelGGL((k_zconv_batch<T>), dim3(ceil_div(Kx, lpb(2 * nz, Kx)), My, nb), dim3(1024),
                     lds, s, beams);
  PIC_TRY(hipGetLastError());
  hipLaunchKernelGGL((k_c2c_y_batch<T, +1, 1>), dim3(ceil_div(Kx, lpb(My, Kx)), nz + 2, nb),
                     dim3(1024), lds, s, beams);
  PIC_TRY(hipGetLastError());
  hipLaunchKernelGGL((k_c2r_x_batch<T>), dim3(ceil_div(ny + 2, lpb(nx, ny + 2)), nz + 2, nb),
                     dim3(1024), lds, s, beams);
  PIC_TRY(hipGetLastError());
  const int64_t ng = (int64_t)nx * ny * nz;
  hipLaunchKernelGGL((k_grad_batch<T>), dim3(grid_for(ng), nb), dim3(256), 0, s, beams);
  return hipGetLastError();
}

template hipError_t launch_batch_green<double>(const BeamDev*, int, const BatchDims&, hipStream_t);
template hipError_t launch_batch_green<float>(const BeamDev*, int, const BatchDims&, hipStream_t);
template hipError_t launch_batch_solve<double>(const BeamDev*, int, const BatchDims&, hipStream_t);
template hipError_t launch_batch_solve<float>(const BeamDev*, int, const BatchDims&, hipStream_t);

template hipError_t launch_green_spectrum<double>(const Geom*, const FftPlan&, int, int, int,
                                                  double2*, double*, double*, hipStream_t);
template hipError_t launch_green_dh_spectra<double>(const Geom*, const FftPlan&, int, int, int,
                                                    bool, double2*, double*, double*, hipStream_t);
template hipError_t launch_green_dh_spectra<float>(const Geom*, const FftPlan&, int, int, int,
                                                   bool, double2*, double*, float*, hipStream_t);
template hipError_t launch_green_spectrum<float>(const Geom*, const FftPlan&, int, int, int,
                                                 double2*, double*, float*, hipStream_t);
template hipError_t launch_solve<double>(const Geom*, const FftPlan&, int, int, int,
                                         const double*, void*, const double*, double*, double*,
                                         hipStream_t);
template hipError_t launch_solve<float>(const Geom*, const FftPlan&, int, int, int, const float*,
                                        void*, const float*, float*, float*, hipStream_t);

}  // namespace pic
