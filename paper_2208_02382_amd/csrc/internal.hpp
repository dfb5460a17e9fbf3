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

// One transform length and its radices (4s, then a 2, then 3s, in order of use).
struct FftAxis {
  int M;
  int nrad;
  int rad[12];
};

// FFT plan for the three padded axes.
struct FftPlan {
  FftAxis full[3];       // padded lengths M_a = 2 n_a
  FftAxis half_x;        // n_x: the complex transform inside the real x transforms
  const double2* tw[3];  // exp(-2 pi i t/M_a), t = 0..M_a-1 (float64 master tables)
  const float2* twf[3];  // the same rounded to float32
};

// 6x6 lower-triangular Cholesky factor (row-major, upper part zero).
struct Chol {
  double L[36];
};

constexpr int kMaxTiles = 4096;       // tiles of the per-step particle binning
// Dynamic LDS of the binned deposit's and gather's tile windows: gfx950 gives a workgroup up to
// 160 KB, of which 4 KB are left to the kernels' static LDS (above 64 KB a kernel's
// dynamic-LDS attribute is raised before the launch, see lds_optin)
constexpr size_t kMaxLdsBytes = 163840 - 4096;
constexpr int kMaxThreads = 1024;     // workgroup size limit of the binned deposit and gather

// Binning plan: tiles of T[a] cells along each axis (NT[a] tiles), work chunks of at most
// `chunk` particles for the tiled deposit.
struct SortPlan {
  int T[3];
  int NT[3];
  int ntiles;
  int chunk;
  int64_t max_chunks;
  int blocks;       // workgroups of the binned deposit and gather
  int threads;      // threads per workgroup of the binned gather (64..1024)
  int dep_threads;  // threads per workgroup of the binned charge deposit (64..1024)
};

// One half of a lattice slice's linear map (applied by apply_half, device_common.hpp).  A slice
// is the split-operator step: first half map, space-charge kick over L, second half map.
constexpr int kHalfDrift = 0;      // x += l px, y += l py, z += l delta / gamma^2
constexpr int kHalfThinDrift = 1;  // thin quad k (px -= k x, py += k y), then the drift l
constexpr int kHalfMatrix = 2;     // (x, px) <- mx (x, px), (y, py) <- my (y, py),
                                   // z += mz delta / gamma^2 (thick quadrupole)
struct HalfMap {
  int type;
  int pad;
  double k, ell;          // kHalfDrift, kHalfThinDrift
  double mx[4], my[4];    // kHalfMatrix, row-major
  double mz;              // kHalfMatrix
};
struct SliceDev {
  double L;               // kick length
  HalfMap first, second;
};

// A slice as the reverse sweep sees it: its half maps and kick length, the lattice element
// whose strength it uses (dJ/dk slot), and the strength derivatives of its half maps.
constexpr int kDkNone = 0;    // no strength (drift)
constexpr int kDkThin = 1;    // thin quad inside the first half map (kHalfThinDrift)
constexpr int kDkMatrix = 2;  // quadrupole half maps: d(first)/dk and d(second)/dk (second)^-1
struct AdjSlice {
  HalfMap first, second;
  double L;
  int elem;
  int dk_kind;
  double dfx[4], dfy[4];  // d(first)/dk per plane, row-major (kDkMatrix)
  double dgx[4], dgy[4];  // d(second)/dk times the inverse of second, per plane (kDkMatrix)
};

// Per-beam device descriptor of a batch: every batched kernel takes its beam from the grid
// (blockIdx.y, or blockIdx.z for the two-dimensional FFT passes) and reads this.
struct BeamDev {
  Consts c;
  SortPlan sp;
  FftPlan plan;
  double* X;            // the caller's phase space
  double* XA;           // workspace copies (step j reads XA for even j, XB for odd j)
  double* XB;
  uint32_t* idA;
  uint32_t* idB;
  uint32_t* keys;
  uint32_t* perm;       // the ranking after a call's first step: slot -> index in the step's input
  uint32_t* hist;
  uint32_t* cursor;
  int4* chunks;
  uint32_t* nchunks;
  Geom* geom;
  Box* box;
  void* rho;
  void* phi;
  void* E;
  void* W;
  double* Gd;
  void* Gh;
  double2* corners;
  const SliceDev* slices;  // lattice of this beam, one entry per slice (cycled over the steps)
  int n_slices;
  int pad;
  unsigned long long* tacc;  // per-tile integer charge windows and their exponents
  int* tscale;
};

constexpr int kReduceBlocks = 1024;   // partial sums for the moments reduction
constexpr int kAdjBlocks = 1024;      // grid of the reverse-sweep particle kernels
constexpr int kMaxLattice = 1024;     // lattice elements of the reverse sweep
constexpr int kMomentSlots = 27;      // 6 sums + 21 centred products

// record a failure as the calling thread's pic_last_error() message and return `status`
// (api.cpp); the HIP form also clears the runtime's sticky error of a rejected call
int record_failure(int status, const char* msg);
int record_hip_failure(hipError_t e, const char* where);

// return a failing hipError_t from the enclosing launcher
#define PIC_TRY(x)                   \
  do {                               \
    hipError_t e_ = (x);             \
    if (e_ != hipSuccess) return e_; \
  } while (0)

// ---- launch wrappers (particles.hip)
hipError_t launch_box_reset(Box* box, hipStream_t s);
hipError_t launch_box(const double* X, int64_t n, Box* box, hipStream_t s);
hipError_t launch_geometry(const Box* box, Geom* g, Consts c, hipStream_t s);
hipError_t launch_init_normals(double* X, const double* xi, int64_t n, Chol L, hipStream_t s);
// dist 0: Gaussian with a uniform halo of n_halo trailing particles; 1: Waterbag (n_halo 0)
hipError_t launch_init_philox(double* X, int64_t n, int64_t n_halo, uint64_t seed, Chol L,
                              int dist, hipStream_t s);
hipError_t launch_clear_status(Geom* g, hipStream_t s);
template <typename T>
hipError_t launch_gather(const double* X, const Geom* g, const T* E, T* Ep, Consts c,
                         hipStream_t s);
template <typename T>
hipError_t launch_push(double* X, int kind, double value, const T* Ep, Consts c, hipStream_t s);
template <typename T>
hipError_t launch_gkd(double* X, const Geom* g, const T* E, double L, const HalfMap& second,
                      int has_next, const HalfMap& first_next, Consts c, Box* box, hipStream_t s);
hipError_t launch_moments(const double* X, int64_t n, double* partial, double* out,
                          hipStream_t s);
template <typename T>
hipError_t launch_zero(T* p, int64_t count, hipStream_t s);

// ---- sort.hip
// nodes of one tile's deposit window, (T_x + S)(T_y + S)(T_z + S)
inline int64_t tile_window_nodes(const SortPlan& sp, int S) {
  return (int64_t)(sp.T[0] + S) * (sp.T[1] + S) * (sp.T[2] + S);
}
// tile[a], chunk, blocks: 0 selects the default
SortPlan make_sort_plan(int nx, int ny, int nz, int64_t n, const int tile[3], int chunk,
                        int blocks, int threads, int deposit_threads = 0);
// A = the first half map of X with the box of its positions; idA (if given) = ids_in, or the
// indices 0..n-1 when ids_in is nullptr
hipError_t launch_prologue(const double* X, double* A, uint32_t* idA, const uint32_t* ids_in,
                           const HalfMap& first, Consts c, Box* box, hipStream_t s);
hipError_t launch_bin(const double* A, const uint32_t* idA, const Geom* g, Consts c,
                      const SortPlan& sp, uint32_t* keys, uint32_t* hist, uint32_t* cursor,
                      int4* chunks, uint32_t* nchunks, double* B, uint32_t* idB, bool staged,
                      hipStream_t s);
// keys and work list as launch_bin, then only the ranking: perm[slot] = index in A
hipError_t launch_bin_perm(const double* A, const Geom* g, Consts c, const SortPlan& sp,
                           uint32_t* keys, uint32_t* hist, uint32_t* cursor, int4* chunks,
                           uint32_t* nchunks, uint32_t* perm, hipStream_t s);
// perm == nullptr: B is in slot order; else slot i reads particle perm[i] of B.  Each tile's
// window is summed exactly as integers in tacc (ntiles * (T+S)^3 64-bit entries, all zero on
// entry and left zero; tscale: kMaxTiles exponents) and the grid rho (zeroed by the caller) is
// formed from them in a fixed order.
template <typename T>
hipError_t launch_deposit_tiles(const double* B, const uint32_t* perm, const Geom* g, Consts c,
                                const SortPlan& sp, const int4* chunks, const uint32_t* nchunks,
                                T* rho, hipStream_t s, unsigned long long* tacc, int* tscale);
// perm == nullptr: B in slot order, updated in place (src, idsrc, iddst unused); else slot i
// reads particle perm[i] of src and id idsrc[perm[i]], and writes slot i of B and iddst
// (src != B, idsrc != iddst; iddst == nullptr: no ids).  diag_out != nullptr: the moments (kMomentSlots doubles) of the
// state after the second half map go to diag_out, summed in the same pass into diag_part
// (sp.blocks * kMomentSlots doubles) about diag_shift (6 doubles, set from diag_prev, the
// previous step's moments, or from the grid centre when diag_prev is nullptr).
template <typename T>
hipError_t launch_gkd_tiles(double* B, const double* src, const uint32_t* perm,
                            const uint32_t* idsrc, uint32_t* iddst, const Geom* g, const T* E,
                            Consts c, const SortPlan& sp, const int4* chunks,
                            const uint32_t* nchunks, double L, const HalfMap& second,
                            int has_next, const HalfMap& first_next, Box* box, hipStream_t s,
                            double* diag_part = nullptr, double* diag_shift = nullptr,
                            const double* diag_prev = nullptr, double* diag_out = nullptr);
// dst = src (bytes, a multiple of 4; both 4-byte aligned) unless the geometry's error flag is set
hipError_t launch_copy_if_ok(const void* src, void* dst, size_t bytes, const Geom* g,
                             hipStream_t s);
// both half maps of a slice without a kick (tracking without space charge)
hipError_t launch_half_maps(double* X, const HalfMap& first, const HalfMap& second, Consts c,
                            hipStream_t s);
// one half map in place and (box != nullptr) the box of the new positions
hipError_t launch_half_box(double* X, const HalfMap& h, Consts c, Box* box, hipStream_t s);
hipError_t launch_unpermute(const double* A, const uint32_t* idA, int64_t n, double* X,
                            uint32_t* keys, uint32_t* hist, uint32_t* cursor, int4* chunks,
                            uint32_t* nchunks, double* B, uint32_t* idB, const Geom* g,
                            hipStream_t s);

// ---- batched tracking (one launch per stage for all beams of a batch)
struct BatchDims {      // grid extents over the beams of a batch
  int64_t max_n;        // largest particle count
  int max_nx, max_ny, max_nz;
  int max_chunks;       // work-list blocks per beam for the tiled deposit and gather
  size_t dep_lds, gkd_lds;
};
hipError_t launch_batch_particles_bin(const BeamDev* beams, int nb, const BatchDims& bd, int shape,
                                      int parity, bool first, hipStream_t s);
// every beam's per-tile integer charge windows set to zero
hipError_t launch_batch_clear_tacc(const BeamDev* beams, int nb, hipStream_t s);
// first: the call's first step, whose binning moved the particles into tile order; later steps
// only rank them, and the deposit and the gather-kick read the step's input through the ranking
template <typename T>
hipError_t launch_batch_deposit(const BeamDev* beams, int nb, const BatchDims& bd, int shape,
                                int parity, bool first, hipStream_t s);
template <typename T>
hipError_t launch_batch_gkd(const BeamDev* beams, int nb, const BatchDims& bd, int shape,
                            int parity, int j, int n_steps, bool first, hipStream_t s);
hipError_t launch_batch_unpermute(const BeamDev* beams, int nb, const BatchDims& bd, int parity,
                                  hipStream_t s);
hipError_t launch_batch_prologue_particles(const BeamDev* beams, int nb, const BatchDims& bd,
                                           hipStream_t s);
hipError_t launch_batch_box_reset(const BeamDev* beams, int nb, hipStream_t s);
hipError_t launch_batch_geometry(const BeamDev* beams, int nb, hipStream_t s);
template <typename T>
hipError_t launch_batch_zero_rho(const BeamDev* beams, int nb, const BatchDims& bd, hipStream_t s);
hipError_t launch_batch_igf(const BeamDev* beams, int nb, int max_nx, int max_ny, int max_nz,
                            hipStream_t s);
template <typename T>
hipError_t launch_batch_green(const BeamDev* beams, int nb, const BatchDims& bd, hipStream_t s);
template <typename T>
hipError_t launch_batch_solve(const BeamDev* beams, int nb, const BatchDims& bd, hipStream_t s);

// ---- adjoint.hip
// dk[sl.elem] += sum_i lam_i . DG Xnext_i (the second half map's strength derivative, from the
// state after it), for quadrupole slices; no-op otherwise
hipError_t launch_adj_dk_second(const double* Xnext, const double* lam, Consts c,
                                const AdjSlice& sl, double* dk_partial, double* dk,
                                hipStream_t s);
// launch_adj_a and launch_adj_stage also find the particles at the box's min and max of the
// kick-point positions (the first index for a tie): their indices into geo[0..5] (x, y, z min,
// then max), ext_partial (12 doubles per block) as scratch
template <typename T>
hipError_t launch_adj_a(const double* X, double* lam, const Geom* g, Consts c,
                        const AdjSlice& sl, T* e, double* ext_partial, double* geo,
                        hipStream_t s);
hipError_t launch_adj_stage(const double* X, double* lam, const Geom* g, Consts c,
                            const AdjSlice& sl, double* P, double* ext_partial, double* geo,
                            hipStream_t s);
// out[c] = sum_i a[c stride + i] b[c stride + i], i < count, c < ncomp (at most 64), in a fixed
// order; partial holds ncomp doubles per block
template <typename T>
hipError_t launch_grid_dot(const T* a, const T* b, int64_t count, int ncomp, int64_t stride,
                           double* partial, double* out, hipStream_t s);
// the geometry's terms of a reverse step from geo (see adjoint.hip) into lam and dk
hipError_t launch_adj_geom(const double* X, double* lam, const Geom* g, Consts c,
                           const AdjSlice& sl, const double* geo, double* dk, hipStream_t s);
// binned vector deposit; an error if the three float64 windows exceed the LDS a workgroup may use
template <typename T>
hipError_t launch_vdeposit_tiles(const double* B, const Geom* g, Consts c, const SortPlan& sp,
                                 const int4* chunks, const uint32_t* nchunks, T* e,
                                 hipStream_t s);
template <typename T>
hipError_t launch_adj_div(const Geom* g, const T* e, T* psi, int nx, int ny, int nz,
                          hipStream_t s);
// also the per-block sums of g_a and g_a u_a (6 kAdjBlocks doubles of geo_partial) into
// geo[6..11]
template <typename T>
hipError_t launch_adj_b(const double* X, double* lam, const Geom* g, Consts c, const AdjSlice& sl,
                        const T* E, const T* chi, double* dk_partial, double* dk,
                        double* geo_partial, double* geo, hipStream_t s);
// (sigma_x, sigma_y, eps_x, eps_y) from the moments mom (mean 6, covariance upper 21) into
// the device array out_m[4]
hipError_t launch_objective(const double* mom, double* out_m, hipStream_t s);
hipError_t launch_obj_grad(const double* X, int64_t n, const double* mom, const double w[4],
                           double* lam, double* out_m, hipStream_t s);
hipError_t launch_dL(const double* lam, const double* xi, int64_t n, double* partial, double* out,
                     hipStream_t s);

// ---- igf.hip
// the kernels' h-derivatives on the octant: 3 (potential, dGbar/dh_b) or 9 (field,
// dKbar_a/dh_b at 3 a + b) corner arrays dc and cell arrays gd
hipError_t launch_igf_dh(const Geom* g, int nx, int ny, int nz, bool field, double2* dc,
                         double* gd, hipStream_t s);
// their spectra, scaled as the Green spectrum: gh[b] (potential) or gh[3 b + a] (field)
template <typename T>
hipError_t launch_green_dh_spectra(const Geom* g, const FftPlan& p, int nx, int ny, int nz,
                                   bool field, double2* dc, double* gd, T* gh, hipStream_t s);
// the field kernels: corner values of H_x, H_y, H_z (3 (nx+2)(ny+2)(nz+2) double pairs) and
// the three octant arrays Kbar_a (3 (nx+1)(ny+1)(nz+1) doubles)
hipError_t launch_igf_field(const Geom* g, int nx, int ny, int nz, double2* hc, double* gd3,
                            hipStream_t s);
// spectra of the three field kernels (gh3: 3 octant arrays, each i times the stored value)
template <typename T>
hipError_t launch_green_field_spectrum(const Geom* g, const FftPlan& p, int nx, int ny, int nz,
                                       double2* hcorners, double* gd3, T* gh3, hipStream_t s);
// E' (3 [nz][ny][nx]) directly from rho with the field spectra; W2: [nz][2 ny][nx+1] complex
// the transposed direct-field solve: chi = -sum_a (Kbar_a * e_a) / (4 pi eps0) on nodes
// 0..n-1 from the three components e[3][nz][ny][nx]; tmp holds 3 nx ny nz values
template <typename T>
hipError_t launch_solve_field_T(const Geom* g, const FftPlan& p, int nx, int ny, int nz,
                                const T* e, void* W, void* W2, const T* gh3, T* tmp, T* chi,
                                hipStream_t s);
template <typename T>
hipError_t launch_solve_field(const Geom* g, const FftPlan& p, int nx, int ny, int nz,
                              const T* rho, void* W, void* W2, const T* gh3, T* E, hipStream_t s);
hipError_t launch_igf_corners(const Geom* g, int nx, int ny, int nz, double2* corners,
                              hipStream_t s);
hipError_t launch_igf_cells(const Geom* g, int nx, int ny, int nz, const double2* corners,
                            double* gd /* (nz+1)(ny+1)(nx+1) */, hipStream_t s);

// ---- fft.hip
hipError_t launch_twiddles(double2* tw, float2* twf, int M, hipStream_t s);
template <typename T>
hipError_t launch_green_spectrum(const Geom* g, const FftPlan& p, int nx, int ny, int nz,
                                 double2* corners, double* gd, T* gh, hipStream_t s);
template <typename T>
hipError_t launch_solve(const Geom* g, const FftPlan& p, int nx, int ny, int nz, const T* rho,
                        void* W, const T* Gh, T* phi, T* E, hipStream_t s);
// chi on nodes 0..n-1 = 1/(4 pi eps0) Gbar * psi for psi on nodes -1..n ([(nz+2)][(ny+2)][(nx+2)])
template <typename T>
hipError_t launch_solve_ghost_source(const Geom* g, const FftPlan& p, int nx, int ny, int nz,
                                     const T* psi, void* W, const T* Gh, T* chi, hipStream_t s);

}  // namespace pic
