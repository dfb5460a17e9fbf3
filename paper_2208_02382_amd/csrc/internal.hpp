// Internal declarations shared by the translation units of libpic.so (host and device).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pic {

// Device-resident geometry of the current step (written by k_geometry, read by every grid or
// stencil kernel).  status != 0 makes every kernel that reads it skip its work.
struct Geom {
  double origin[3];   // lab position of node 0 along x, y, z
  double h[3];        // lab spacings
  double inv_h[3];    // 1/h
  double h_rest[3];   // rest-frame spacings (hx, hy, gamma hz)
  int status;         // 0 = ok, else a pic_status value
  int pad[3];
};

// Box accumulator: min/max of x, y, z in order-preserving uint64 encoding, and a non-finite
// flag.  Reset by k_box_reset before each reduction.
struct Box {
  unsigned long long mn[3];
  unsigned long long mx[3];
  unsigned int nonfinite;
  unsigned int pad[3];
};

// Problem constants passed by value to kernels.
struct Consts {
  int64_t n;
  int nx, ny, nz;
  int shape;           // 1 CIC, 2 TSC
  double gamma;
  double inv_gamma2;   // 1/gamma^2
  double C;            // kick constant qm/(gamma^2 beta^2) [1/V]
  double q_macro;      // charge per macroparticle [C]
};

// Twiddle tables and FFT plan for the three padded axes.
struct FftPlan {
  int M[3];            // padded lengths (x, y, z)
  int nrad[3];
  int rad[3][12];      // radices per axis (4, 2, 3 in that order of use)
  const double2* tw[3];  // exp(-2 pi i t/M), t = 0..M-1 (float64 master tables)
  const float2* twf[3];  // the same rounded to float32
};

// 6x6 lower-triangular Cholesky factor (row-major, upper part zero).
struct Chol {
  double L[36];
};

constexpr int kReduceBlocks = 1024;   // partial sums for the moments reduction
constexpr int kMomentSlots = 27;      // 6 sums + 21 centred products

// ---- launch wrappers (particles.hip)
hipError_t launch_box_reset(Box* box, hipStream_t s);
hipError_t launch_box(const double* X, int64_t n, Box* box, hipStream_t s);
hipError_t launch_geometry(const Box* box, Geom* g, Consts c, hipStream_t s);
hipError_t launch_init_normals(double* X, const double* xi, int64_t n, Chol L, hipStream_t s);
hipError_t launch_init_philox(double* X, int64_t n, int64_t n_halo, uint64_t seed, Chol L,
                              hipStream_t s);
hipError_t launch_clear_status(Geom* g, hipStream_t s);
template <typename T>
hipError_t launch_deposit(const double* X, const Geom* g, T* rho, Consts c, hipStream_t s);
template <typename T>
hipError_t launch_gather(const double* X, const Geom* g, const T* E, T* Ep, Consts c,
                         hipStream_t s);
template <typename T>
hipError_t launch_push(double* X, int kind, double value, const T* Ep, Consts c, hipStream_t s);
hipError_t launch_quad_drift(double* X, double k, double ell, Consts c, Box* box, hipStream_t s);
template <typename T>
hipError_t launch_gkd(double* X, const Geom* g, const T* E, double L, int has_next, double k_next,
                      double half_next, Consts c, Box* box, hipStream_t s);
hipError_t launch_moments(const double* X, int64_t n, double* partial, double* out,
                          hipStream_t s);
template <typename T>
hipError_t launch_zero(T* p, int64_t count, hipStream_t s);

// ---- igf.hip
hipError_t launch_igf_corners(const Geom* g, int nx, int ny, int nz, double2* corners,
                              hipStream_t s);
template <typename T>
hipError_t launch_igf_place(const Geom* g, int nx, int ny, int nz, const double2* corners,
                            void* W /* complex<T> M^3 */, hipStream_t s);

// ---- fft.hip
hipError_t launch_twiddles(double2* tw, float2* twf, int M, hipStream_t s);
template <typename T>
hipError_t launch_green_spectrum(const Geom* g, const FftPlan& p, int nx, int ny, int nz,
                                 double2* corners, void* W, T* Gh, hipStream_t s);
template <typename T>
hipError_t launch_solve(const Geom* g, const FftPlan& p, int nx, int ny, int nz, const T* rho,
                        void* W, const T* Gh, T* phi, T* E, hipStream_t s);

}  // namespace pic
