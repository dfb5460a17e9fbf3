// C ABI of libpic.so: argument validation, workspace layout and the order of kernel launches.
// Every numerical step runs in the HIP kernels of particles.hip, igf.hip and fft.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "../../include/pic.h"
#include "internal.hpp"

using namespace pic;

namespace {

thread_local std::string g_last_error;

pic_status fail(pic_status st, const char* msg) {
  g_last_error = msg;
  return st;
}

pic_status fail_hip(hipError_t e, const char* where) {
  g_last_error = std::string(where) + ": " + hipGetErrorString(e);
  (void)hipGetLastError();  // a rejected call must not fail the thread's next HIP call
  return PIC_EHIP;
}

}  // namespace

namespace pic {
int record_failure(int status, const char* msg) { return fail((pic_status)status, msg); }
int record_hip_failure(hipError_t e, const char* where) { return fail_hip(e, where); }
}  // namespace pic

namespace {

#define HIP_OK(call, where)                       \
  do {                                            \
    hipError_t e_ = (call);                       \
    if (e_ != hipSuccess) return fail_hip(e_, where); \
  } while (0)

// radices of M = 2^a 3^b in order of use: 4s, then a 2, then 3s; 0 on failure
int factor(int M, int rad[12]) {
  int n = 0, m = M;
  while (m % 4 == 0 && n < 12) { rad[n++] = 4; m /= 4; }
  while (m % 2 == 0 && n < 12) { rad[n++] = 2; m /= 2; }
  while (m % 3 == 0 && n < 12) { rad[n++] = 3; m /= 3; }
  if (m != 1) return 0;
  for (int q = n; q < 12; ++q) rad[q] = 1;
  return n;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

struct Layout {
  size_t geom, box, mom_partial, mom_out, tw[3], twf[3], corners, W, Gd, Gh, rho, phi, E;
  size_t hcorners, gd3, gh3, W2;  // direct field only (else 0-byte slots)
  size_t XA, XB, idA, idB, keys, perm, hist, cursor, chunks, nchunks, diag_part, diag_shift;
  size_t tacc, tscale, total;
};

pic_status check_desc(const pic_beam_desc* d) {
  if (!d) return fail(PIC_EINVAL, "NULL description");
  if (d->n < 1) return fail(PIC_EINVAL, "n must be >= 1");
  if (d->n > 0x7fffffffLL) return fail(PIC_EUNSUPPORTED, "n must be < 2^31");
  if (d->shape != 1 && d->shape != 2) return fail(PIC_EINVAL, "shape must be 1 (CIC) or 2 (TSC)");
  if (d->nx < 4 || d->ny < 4 || d->nz < 4) return fail(PIC_EINVAL, "grid needs >= 4 nodes per axis");
  if (!(d->mass_MeV > 0) || !(d->kin_energy_MeV > 0) || !std::isfinite(d->kin_energy_MeV))
    return fail(PIC_EINVAL, "mass and kinetic energy must be positive");
  if (!std::isfinite(d->qm_qeeV) || d->qm_qeeV == 0.0) return fail(PIC_EINVAL, "qm_qeeV must be finite and non-zero");
  if (!std::isfinite(d->charge_C) || d->charge_C < 0) return fail(PIC_EINVAL, "charge_C must be >= 0");
  if (d->grid_fp32 != 0 && d->grid_fp32 != 1) return fail(PIC_EINVAL, "grid_fp32 must be 0 or 1");
  if (d->space_charge != 0 && d->space_charge != 1) return fail(PIC_EINVAL, "space_charge must be 0 or 1");
  int nn[3] = {d->nx, d->ny, d->nz};
  for (int a = 0; a < 3; ++a) {
    int rad[12];
    int M = 2 * nn[a];
    if (M > 512 || factor(M, rad) == 0)
      return fail(PIC_EUNSUPPORTED, "padded FFT length 2*n must be 2^a 3^b and <= 512");
  }
  int64_t ntiles = 1, window = 8;  // the deposit window holds 64-bit fixed-point charges
  for (int a = 0; a < 3; ++a) {
    if (d->tile[a] < 0 || d->tile[a] > nn[a]) return fail(PIC_EINVAL, "tile must be in 0..n_a");
    const int t = d->tile[a] > 0 ? d->tile[a] : std::max(4, (nn[a] + 15) / 16);
    ntiles *= (nn[a] + t - 1) / t;
    window *= t + d->shape;
  }
  if (ntiles > kMaxTiles) return fail(PIC_EINVAL, "tile count must be <= 4096");
  // the deposit's charge window of a tile lives in LDS (156 KB per workgroup)
  if (window > (int64_t)kMaxLdsBytes) return fail(PIC_EINVAL, "tile charge window exceeds the 156 KB of LDS a workgroup may use");
  if (d->chunk != 0 && (d->chunk < 256 || d->chunk > (1 << 20)))
    return fail(PIC_EINVAL, "chunk must be 0 or 256..2^20");
  if (d->blocks < 0 || d->blocks > 65535) return fail(PIC_EINVAL, "blocks must be 0..65535");
  if (d->threads != 0 && (d->threads < 64 || d->threads > kMaxThreads || d->threads % 64 != 0))
    return fail(PIC_EINVAL, "threads must be 0 or a multiple of 64 in 64..1024");
  if (d->deposit_threads != 0 && (d->deposit_threads < 64 || d->deposit_threads > kMaxThreads ||
                                  d->deposit_threads % 64 != 0))
    return fail(PIC_EINVAL, "deposit_threads must be 0 or a multiple of 64 in 64..1024");
  if (d->direct_field != 0 && d->direct_field != 1) return fail(PIC_EINVAL, "direct_field must be 0 or 1");
  return PIC_OK;
}

Layout layout(const pic_beam_desc* d) {
  Layout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  const size_t es = d->grid_fp32 ? 4 : 8;
  const size_t nx = d->nx, ny = d->ny, nz = d->nz;
  // half spectrum of the padded grid: (2 nz)(2 ny)(nx + 1) complex values
  const size_t Wn = 4 * nz * ny * (nx + 1);
  const size_t G3 = (nx + 1) * (ny + 1) * (nz + 1);
  L.geom = take(sizeof(Geom));
  L.box = take(sizeof(Box));
  L.mom_partial = take(sizeof(double) * kReduceBlocks * kMomentSlots);
  L.mom_out = take(sizeof(double) * (kMomentSlots + 4));  // moments, then the objective terms
  int nn[3] = {d->nx, d->ny, d->nz};
  for (int a = 0; a < 3; ++a) L.tw[a] = take(sizeof(double2) * 2 * nn[a]);
  for (int a = 0; a < 3; ++a) L.twf[a] = take(sizeof(float2) * 2 * nn[a]);
  L.corners = take(sizeof(double2) * (nx + 2) * (ny + 2) * (nz + 2));
  L.W = take(2 * es * Wn);
  L.Gd = take(sizeof(double) * G3);
  L.Gh = take(es * G3);
  L.rho = take(es * nx * ny * nz);
  L.phi = take(es * (nx + 2) * (ny + 2) * (nz + 2));
  L.E = take(3 * es * nx * ny * nz);
  // the direct field's kernels: corner values, octant arrays, spectra, second work array
  const size_t df = d->direct_field ? 1 : 0;
  L.hcorners = take(df * 3 * sizeof(double2) * (nx + 2) * (ny + 2) * (nz + 2));
  L.gd3 = take(df * 3 * sizeof(double) * G3);
  L.gh3 = take(df * 3 * es * G3);
  L.W2 = take(df * 2 * es * nz * 2 * ny * (nx + 1));
  // tracking-loop buffers: two sorted copies of the phase space, particle ids, tile keys,
  // the sort permutation, tile histogram / sort cursors and the deposit work list
  const size_t n = (size_t)d->n;
  const SortPlan sp = make_sort_plan(d->nx, d->ny, d->nz, d->n, d->tile, d->chunk, d->blocks,
                                     d->threads);
  L.XA = take(6 * sizeof(double) * n);
  L.XB = take(6 * sizeof(double) * n);
  L.idA = take(sizeof(uint32_t) * n);
  L.idB = take(sizeof(uint32_t) * n);
  L.keys = take(sizeof(uint32_t) * n);
  L.perm = take(sizeof(uint32_t) * n);
  L.hist = take(sizeof(uint32_t) * kMaxTiles);
  L.cursor = take(sizeof(uint32_t) * kMaxTiles);
  L.chunks = take(sizeof(int4) * (size_t)sp.max_chunks);
  L.nchunks = take(sizeof(uint32_t));
  // slice-step diagnostics summed inside the gather-kick: one partial per workgroup, the shift
  L.diag_part = take(sizeof(double) * kMomentSlots * (size_t)sp.blocks);
  L.diag_shift = take(sizeof(double) * 6);
  // the deposit's per-tile integer windows (the order-independent charge grid) and exponents
  L.tacc = take(sizeof(uint64_t) * (size_t)sp.ntiles * tile_window_nodes(sp, d->shape));
  L.tscale = take(sizeof(int) * kMaxTiles);
  L.total = off;
  return L;
}

}  // namespace

// HIP event pairs around the stages of pic_track_n_steps (enabled by pic_profile_start)
struct StageProfiler {
  bool on = false;
  std::vector<hipEvent_t> pool;   // created on demand, reused across reads
  std::vector<int> stage;         // stage of pair k (events 2k, 2k+1)
  size_t used = 0;                // pairs recorded since the last start
  hipError_t begin(int st, hipStream_t s) {
    if (!on) return hipSuccess;
    while (pool.size() < 2 * (used + 1)) {
      hipEvent_t e;
      hipError_t r = hipEventCreate(&e);
      if (r != hipSuccess) return r;
      pool.push_back(e);
    }
    if (stage.size() < used + 1) stage.resize(used + 1);
    stage[used] = st;
    return hipEventRecord(pool[2 * used], s);
  }
  hipError_t end(hipStream_t s) {
    if (!on) return hipSuccess;
    hipError_t r = hipEventRecord(pool[2 * used + 1], s);
    ++used;
    return r;
  }
  ~StageProfiler() {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
};

// The end of the last work a handle enqueued, so that its teardown can wait for it before it
// destroys the streams, events and graph executables that work may still use.  HIP does not
// promise that destroying a graph executable or an event in flight is safe.
struct DoneEvent {
  hipEvent_t ev = nullptr;
  bool pending = false;
  void mark(hipStream_t s) {
    if (ev && hipEventRecord(ev, s) == hipSuccess) pending = true;
  }
  void wait() {
    if (ev && pending) (void)hipEventSynchronize(ev);
    pending = false;
  }
};

struct pic_beam_s {
  pic_beam_desc d;
  StageProfiler prof;
  double* X;
  char* work;
  Layout L;
  Consts c;
  FftPlan plan;
  Geom* geom;
  Box* box;
  double* mom_partial;
  double* mom_out;
  double* diag_part;   // per-workgroup moment sums of the fused slice-step diagnostics
  double* diag_shift;
  unsigned long long* tacc;  // per-tile integer charge windows (zero between deposits)
  int* tscale;
  double2* corners;
  void* W;
  double* Gd;
  void* Gh;
  void* rho;
  void* phi;
  void* E;
  double2* hcorners;  // direct field (pic_beam_desc.direct_field)
  double* gd3;
  void* gh3;
  void* W2;
  SortPlan sp;
  double* XA;
  double* XB;
  uint32_t* idA;
  uint32_t* idB;
  uint32_t* keys;
  uint32_t* perm;
  uint32_t* hist;
  uint32_t* cursor;
  int4* chunks;
  uint32_t* nchunks;
  // X is in the tile order a pic_track_n_steps_binned call left it in (the next binned call
  // then only ranks on its first step); the initialisations reset it
  bool x_binned = false;
  // the Green spectrum of a step runs on `aux`, concurrently with the binning and deposit
  hipStream_t aux = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  DoneEvent done;  // recorded on the caller's stream at the end of every enqueuing call
  ~pic_beam_s() {
    // the caller's stream may still wait on ev_join and run kernels of this handle: wait for
    // the last enqueued call and for the auxiliary stream before releasing them
    done.wait();
    if (aux) (void)hipStreamSynchronize(aux);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (done.ev) (void)hipEventDestroy(done.ev);
    if (aux) (void)hipStreamDestroy(aux);
  }
};

// auxiliary stream (default priority), fork / join events and the completion event
hipError_t make_aux(hipStream_t* aux, hipEvent_t* fork, hipEvent_t* join, hipEvent_t* done) {
  hipError_t e = hipStreamCreateWithFlags(aux, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(join, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(done, hipEventDisableTiming);
  return e;
}

// records the handle's completion event on the call's stream when the call returns (whatever
// it returns: a failed call may have enqueued part of its work)
struct MarkDone {
  DoneEvent& d;
  hipStream_t s;
  ~MarkDone() { d.mark(s); }
};

namespace {

hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

pic_status device_status(int st) {
  if (st == 0) return PIC_OK;
  if (st == PIC_EINTERNAL) return fail(PIC_EINTERNAL, "device detected an inconsistent particle binning");
  return fail(PIC_EDOMAIN, "device flagged a non-finite coordinate or a zero-extent box");
}

bool cholesky6(const double* A, Chol& out) {
  double L[36] = {0};
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j)
      if (!std::isfinite(A[i * 6 + j]) || std::fabs(A[i * 6 + j] - A[j * 6 + i]) >
                                               1e-12 * (std::fabs(A[i * 6 + j]) + std::fabs(A[j * 6 + i])))
        return false;
  for (int j = 0; j < 6; ++j) {
    double s = A[j * 6 + j];
    for (int k = 0; k < j; ++k) s -= L[j * 6 + k] * L[j * 6 + k];
    if (!(s > 0)) return false;
    L[j * 6 + j] = std::sqrt(s);
    for (int i = j + 1; i < 6; ++i) {
      double t = A[i * 6 + j];
      for (int k = 0; k < j; ++k) t -= L[i * 6 + k] * L[j * 6 + k];
      L[i * 6 + j] = t / L[j * 6 + j];
    }
  }
  std::memcpy(out.L, L, sizeof(L));
  return true;
}

#define STAGE(b, st, s, call, where)            \
  do {                                          \
    HIP_OK((b)->prof.begin((st), (s)), "profile"); \
    HIP_OK((call), (where));                    \
    HIP_OK((b)->prof.end(s), "profile");        \
  } while (0)

// the kernel spectra of the step's geometry: the potential's, or the three field kernels'
template <typename T>
hipError_t green_spectra(pic_beam b, hipStream_t s) {
  if (b->d.direct_field)
    return launch_green_field_spectrum<T>(b->geom, b->plan, b->d.nx, b->d.ny, b->d.nz,
                                          b->hcorners, b->gd3, (T*)b->gh3, s);
  return launch_green_spectrum<T>(b->geom, b->plan, b->d.nx, b->d.ny, b->d.nz, b->corners,
                                  b->Gd, (T*)b->Gh, s);
}

template <typename T>
pic_status green_and_solve(pic_beam b, const T* rho, T* phi, T* E, hipStream_t s,
                           bool green = true) {
  if (green)
    STAGE(b, PIC_STAGE_GREEN, s, green_spectra<T>(b, s), "green spectrum");
  if (b->d.direct_field)
    STAGE(b, PIC_STAGE_SOLVE, s,
          launch_solve_field<T>(b->geom, b->plan, b->d.nx, b->d.ny, b->d.nz, rho, b->W, b->W2,
                                (const T*)b->gh3, E, s),
          "field solve");
  else
    STAGE(b, PIC_STAGE_SOLVE, s,
          launch_solve<T>(b->geom, b->plan, b->d.nx, b->d.ny, b->d.nz, rho, b->W,
                          (const T*)b->Gh, phi, E, s),
          "poisson solve");
  return PIC_OK;
}

// ---- lattice slices (element kinds of pic_element)
HalfMap half_drift(double ell) {
  HalfMap h{};
  h.type = kHalfDrift;
  h.ell = ell;
  return h;
}

HalfMap half_thin(double k, double ell) {
  HalfMap h{};
  h.type = kHalfThinDrift;
  h.k = k;
  h.ell = ell;
  return h;
}

// (x, px) map of a quadrupole of strength k over length s: focusing for k > 0
void quad_2x2(double k, double s, double m[4]) {
  if (k > 0) {
    const double r = std::sqrt(k), c = std::cos(r * s), sn = std::sin(r * s);
    m[0] = c; m[1] = sn / r; m[2] = -r * sn; m[3] = c;
  } else if (k < 0) {
    const double r = std::sqrt(-k), c = std::cosh(r * s), sn = std::sinh(r * s);
    m[0] = c; m[1] = sn / r; m[2] = r * sn; m[3] = c;
  } else {
    m[0] = 1.0; m[1] = s; m[2] = 0.0; m[3] = 1.0;
  }
}

HalfMap half_quad(double k, double ell) {
  HalfMap h{};
  h.type = kHalfMatrix;
  quad_2x2(k, ell, h.mx);
  quad_2x2(-k, ell, h.my);
  h.mz = ell;
  return h;
}

// One tracking step per slice: THIN is the thin quad k followed by the space-charge drift ds
// (one slice); DRIFT and QUAD elements are cut into nslice slices of ds / nslice, each the
// element map over half the slice, the kick over the slice, the map over the other half.
pic_status expand_lattice(const pic_element* lat, int n_el, std::vector<SliceDev>& out) {
  out.clear();
  for (int q = 0; q < n_el; ++q) {
    const pic_element& e = lat[q];
    if (!std::isfinite(e.k) || !std::isfinite(e.ds) || e.ds < 0.0)
      return fail(PIC_EINVAL, "lattice element needs finite k and ds >= 0");
    if (e.kind == PIC_ELEM_THIN) {
      SliceDev sl{};
      sl.L = e.ds;
      sl.first = half_thin(e.k, 0.5 * e.ds);
      sl.second = half_drift(0.5 * e.ds);
      out.push_back(sl);
    } else if (e.kind == PIC_ELEM_DRIFT || e.kind == PIC_ELEM_QUAD) {
      if (e.nslice < 1 || e.nslice > 1000000) return fail(PIC_EINVAL, "nslice must be 1..1e6");
      const double ell = e.ds / e.nslice;
      SliceDev sl{};
      sl.L = ell;
      sl.first = e.kind == PIC_ELEM_QUAD ? half_quad(e.k, 0.5 * ell) : half_drift(0.5 * ell);
      sl.second = sl.first;
      for (int r = 0; r < e.nslice; ++r) out.push_back(sl);
    } else {
      return fail(PIC_EINVAL, "unknown lattice element kind");
    }
  }
  return PIC_OK;
}

// the deposit's per-tile integer windows start at zero (each deposit leaves them zero; a call
// interrupted by a device error may not)
hipError_t clear_tacc(pic_beam b, hipStream_t s) {
  return launch_zero<double>((double*)b->tacc,
                             (int64_t)b->sp.ntiles * tile_window_nodes(b->sp, b->d.shape), s);
}

// Green spectrum of the current geometry on the auxiliary stream (joined before the solve)
template <typename T>
pic_status fork_green(pic_beam b, hipStream_t s) {
  HIP_OK(hipEventRecord(b->ev_fork, s), "fork");
  HIP_OK(hipStreamWaitEvent(b->aux, b->ev_fork, 0), "fork");
  STAGE(b, PIC_STAGE_GREEN, b->aux, green_spectra<T>(b, b->aux), "green spectrum");
  HIP_OK(hipEventRecord(b->ev_join, b->aux), "join");
  return PIC_OK;
}

// diag: nullptr, or a device array that receives the moments (kMomentSlots doubles) of the
// particles at the end of every step.  The binned gather-kick sums them in the same pass, about
// the previous step's means; the unbinned fallback stops at the end of the step and separate
// passes take the moments and apply the next step's first half map.
// binned: leave X in the step's tile order instead of returning it to the caller's order; the
// last gather-kick writes X (and ids_io, the caller's labels, when given) directly.  With
// first_ranked (X is in the tile order of a previous binned call) the first step only ranks
// instead of moving the particles into tile order.
template <typename T>
pic_status track_sc(pic_beam b, const std::vector<SliceDev>& sl, int n_steps, double* diag,
                    hipStream_t s, bool binned = false, uint32_t* ids_io = nullptr,
                    bool first_ranked = false) {
  const int ns = (int)sl.size();
  const int64_t ng = (int64_t)b->d.nx * b->d.ny * b->d.nz;
  double* A = b->XA;
  double* B = b->XB;
  // without labels a binned call carries no ids
  const bool ids = !binned || ids_io;
  uint32_t* idA = ids ? b->idA : nullptr;
  uint32_t* idB = ids ? b->idB : nullptr;
  HIP_OK(launch_box_reset(b->box, s), "box reset");
  HIP_OK(clear_tacc(b, s), "clear");
  STAGE(b, PIC_STAGE_PROLOGUE, s,
        launch_prologue(b->X, A, idA, binned ? ids_io : nullptr, sl[0].first, b->c, b->box, s),
        "prologue");
  // the E' window of a tile must fit the LDS a workgroup may use
  const size_t win_bytes = 3 * sizeof(T) * (size_t)(b->sp.T[0] + b->d.shape) *
                           (b->sp.T[1] + b->d.shape) * (b->sp.T[2] + b->d.shape);
  const bool tiles = win_bytes <= kMaxLdsBytes;
  for (int j = 0; j < n_steps; ++j) {
    const SliceDev& e = sl[j % ns];
    HIP_OK(b->prof.begin(PIC_STAGE_GEOMETRY, s), "profile");
    HIP_OK(launch_geometry(b->box, b->geom, b->c, s), "geometry");
    HIP_OK(launch_zero<T>((T*)b->rho, ng, s), "zero rho");
    HIP_OK(b->prof.end(s), "profile");
    pic_status st = fork_green<T>(b, s);
    if (st != PIC_OK) return st;
    // After the first step A is in the previous step's tile order: only the ranking is
    // written, and the gather-kick moves the particles (A -> B) while it updates them.  The
    // first step moves the caller's order into tile order (A -> B) and updates B in place.
    const bool permuted = tiles && (j > 0 || first_ranked);
    if (permuted)
      STAGE(b, PIC_STAGE_BIN, s,
            launch_bin_perm(A, b->geom, b->c, b->sp, b->keys, b->hist, b->cursor, b->chunks,
                            b->nchunks, b->perm, s),
            "binning");
    else
      STAGE(b, PIC_STAGE_BIN, s,
            launch_bin(A, idA, b->geom, b->c, b->sp, b->keys, b->hist, b->cursor, b->chunks,
                       b->nchunks, B, idB, j == 0, s),
            "binning");
    const double* P = permuted ? A : B;  // particles the deposit reads (through perm)
    STAGE(b, PIC_STAGE_DEPOSIT, s,
          launch_deposit_tiles<T>(P, permuted ? b->perm : nullptr, b->geom, b->c, b->sp,
                                  b->chunks, b->nchunks, (T*)b->rho, s, b->tacc, b->tscale),
          "deposit");
    HIP_OK(hipStreamWaitEvent(s, b->ev_join, 0), "join");
    st = green_and_solve<T>(b, (const T*)b->rho, (T*)b->phi, (T*)b->E, s, false);
    if (st != PIC_OK) return st;
    const int more = j + 1 < n_steps;
    const int has_next = more && (tiles || !diag);  // fuse the next step's first half map
    double* diag_j = diag ? diag + (size_t)kMomentSlots * j : nullptr;
    const SliceDev& nx = sl[(j + 1) % ns];
    if (has_next) HIP_OK(launch_box_reset(b->box, s), "box reset");
    // a binned call's last gather-kick writes the caller's arrays (it always reads A through
    // the ranking, so X is written only if no step has flagged an error)
    const bool to_caller = binned && permuted && !more;
    double* out = to_caller ? b->X : B;
    uint32_t* id_out = to_caller ? ids_io : idB;
    if (tiles)
      STAGE(b, PIC_STAGE_GKD, s,
            launch_gkd_tiles<T>(out, permuted ? A : nullptr, permuted ? b->perm : nullptr,
                                permuted ? idA : nullptr, permuted ? id_out : nullptr, b->geom,
                                (const T*)b->E, b->c, b->sp, b->chunks, b->nchunks, e.L,
                                e.second, has_next, nx.first, b->box, s, b->diag_part,
                                b->diag_shift, j > 0 && diag_j ? diag_j - kMomentSlots : nullptr,
                                diag_j),
            "gather-kick-drift");
    else
      STAGE(b, PIC_STAGE_GKD, s,
            launch_gkd<T>(B, b->geom, (const T*)b->E, e.L, e.second, has_next, nx.first, b->c,
                          b->box, s),
            "gather-kick-drift");
    if (diag && !tiles) {  // moments at the end of the step, then the next first half map
      HIP_OK(launch_moments(B, b->c.n, b->mom_partial, diag_j, s), "diagnostics");
      if (more) {
        HIP_OK(launch_box_reset(b->box, s), "box reset");
        HIP_OK(launch_half_box(B, nx.first, b->c, b->box, s), "diagnostics");
      }
    }
    // B holds the updated particles in slot order
    double* tX = A; A = B; B = tX;
    uint32_t* tI = idA; idA = idB; idB = tI;
  }
  if (binned) {
    // a last step that did not write X (a one-step call that moved the particles, or the
    // gather's global-load fallback) leaves the state in A: copied in slot order
    const bool last_to_caller = tiles && (n_steps > 1 || first_ranked);
    if (!last_to_caller) {
      HIP_OK(launch_copy_if_ok(A, b->X, 6 * sizeof(double) * (size_t)b->c.n, b->geom, s),
             "binned copy");
      if (ids_io)
        HIP_OK(launch_copy_if_ok(idA, ids_io, sizeof(uint32_t) * (size_t)b->c.n, b->geom, s),
               "binned copy");
    }
    return PIC_OK;
  }
  STAGE(b, PIC_STAGE_UNPERMUTE, s,
        launch_unpermute(A, idA, b->c.n, b->X, b->keys, b->hist, b->cursor, b->chunks,
                         b->nchunks, B, idB, b->geom, s),
        "unpermute");
  return PIC_OK;
}

// ---- reverse sweep workspace (caller-owned, see pic_adjoint_workspace_bytes)
struct AdjLayout {
  size_t geoms, ckpt, segX, segE, segG, segQ, e, psi, chi, chi2, stage, dk, dk_part, dL_part,
      small;
  size_t ext_part, geo_part, dot_part, geo, dc, dgd, dgh, total;
  int nseg;
};

constexpr size_t kGeomSlot = 128;  // bytes per stored per-step geometry

AdjLayout adj_layout(const pic_beam_desc* d, int n_steps, int ck) {
  AdjLayout A;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  const size_t es = d->grid_fp32 ? 4 : 8;
  const size_t n = (size_t)d->n, nx = d->nx, ny = d->ny, nz = d->nz;
  const size_t ng = nx * ny * nz, G3 = (nx + 1) * (ny + 1) * (nz + 1);
  A.nseg = (n_steps + ck - 1) / ck;
  A.geoms = take(kGeomSlot * (size_t)n_steps);
  A.ckpt = take(6 * sizeof(double) * n * (size_t)A.nseg);
  A.segX = take(6 * sizeof(double) * n * (size_t)ck);
  A.segE = take(3 * es * ng * (size_t)ck);
  A.segG = take(es * G3 * (size_t)ck * (d->direct_field ? 3 : 1));  // the step's kernel spectra
  A.segQ = take(es * ng * (size_t)ck);                                // the step's charge grid
  A.e = take(3 * es * ng);
  A.psi = take(es * (nx + 2) * (ny + 2) * (nz + 2));
  A.chi = take(es * ng);
  A.chi2 = take(es * ng);
  // the geometry's terms: the kernels' h-derivatives (3 for the potential, 9 for the field:
  // corner values, octant cells, spectra), reduction partials and the per-step sums
  const size_t nf = d->direct_field ? 9 : 3;
  A.dc = take(2 * sizeof(double) * (nx + 2) * (ny + 2) * (nz + 2) * nf);
  A.dgd = take(sizeof(double) * G3 * nf);
  A.dgh = take(es * G3 * nf);
  A.ext_part = take(sizeof(double) * 12 * kAdjBlocks);
  A.geo_part = take(sizeof(double) * 6 * kAdjBlocks);
  A.dot_part = take(sizeof(double) * 3 * kAdjBlocks);
  A.geo = take(sizeof(double) * 32);
  A.stage = take(6 * sizeof(double) * n);
  A.dk = take(sizeof(double) * kMaxLattice);
  A.dk_part = take(sizeof(double) * kAdjBlocks);
  A.dL_part = take(sizeof(double) * 36 * kAdjBlocks);
  A.small = take(sizeof(double) * 64);  // out moments (4) and dJ/dL (36)
  A.total = off;
  static_assert(sizeof(Geom) <= kGeomSlot, "geometry slot too small");
  return A;
}

// d/dk of quad_2x2(k, s), entry by entry: closed forms for |k| s^2 >= 0.1, else the term-by-term
// derivative of the power series in k of cos(sqrt(k) s), sin(sqrt(k) s)/sqrt(k) and
// -sqrt(k) sin(sqrt(k) s), valid for either sign of k
void quad_2x2_dk(double k, double s, double d[4]) {
  if (std::fabs(k) * s * s >= 0.1) {
    const double r = std::sqrt(std::fabs(k));
    if (k > 0) {
      const double c = std::cos(r * s), sn = std::sin(r * s);
      d[0] = d[3] = -s * sn / (2.0 * r);
      d[1] = s * c / (2.0 * k) - sn / (2.0 * r * r * r);
      d[2] = -sn / (2.0 * r) - 0.5 * s * c;
    } else {
      const double c = std::cosh(r * s), sn = std::sinh(r * s);
      d[0] = d[3] = -s * sn / (2.0 * r);
      d[1] = s * c / (2.0 * k) + sn / (2.0 * r * r * r);
      d[2] = -sn / (2.0 * r) - 0.5 * s * c;
    }
    return;
  }
  // d00 = sum_{m>=1} m (-1)^m k^(m-1) s^2m / (2m)!, d01 likewise with s^(2m+1) / (2m+1)!,
  // d10 = -sum_{m>=0} (m+1) (-1)^m k^m s^(2m+1) / (2m+1)!
  double d00 = 0.0, d01 = 0.0, d10 = -s;
  double f2 = 1.0, f3 = 1.0;  // (2m)!, (2m+1)!
  double km1 = 1.0;           // k^(m-1)
  double s2m = 1.0;           // s^2m
  for (int m = 1; m <= 15; ++m) {
    f2 *= (2.0 * m - 1.0) * (2.0 * m);
    f3 *= (2.0 * m) * (2.0 * m + 1.0);
    s2m *= s * s;
    const double sgn = (m & 1) ? -1.0 : 1.0;
    d00 += m * sgn * km1 * s2m / f2;
    d01 += m * sgn * km1 * s2m * s / f3;
    d10 -= (m + 1) * sgn * (km1 * k) * s2m * s / f3;
    km1 *= k;
  }
  d[0] = d[3] = d00;
  d[1] = d01;
  d[2] = d10;
}

// the reverse sweep's view of a lattice: one AdjSlice per slice, as expand_lattice cuts it,
// with the element index and the strength derivatives of the half maps
pic_status expand_adjoint(const pic_element* lat, int n_el, std::vector<AdjSlice>& out) {
  std::vector<SliceDev> sl;
  const pic_status st = expand_lattice(lat, n_el, sl);
  if (st != PIC_OK) return st;
  out.clear();
  size_t j = 0;
  for (int q = 0; q < n_el; ++q) {
    const pic_element& e = lat[q];
    const int count = e.kind == PIC_ELEM_THIN ? 1 : e.nslice;
    for (int r = 0; r < count; ++r, ++j) {
      AdjSlice a{};
      a.first = sl[j].first;
      a.second = sl[j].second;
      a.L = sl[j].L;
      a.elem = q;
      if (e.kind == PIC_ELEM_THIN) {
        a.dk_kind = kDkThin;
      } else if (e.kind == PIC_ELEM_QUAD) {
        a.dk_kind = kDkMatrix;
        const double hs = 0.5 * sl[j].L;
        double dmy[4];
        quad_2x2_dk(e.k, hs, a.dfx);
        quad_2x2_dk(-e.k, hs, dmy);
        for (int t = 0; t < 4; ++t) a.dfy[t] = -dmy[t];  // the y plane sees -k
        // d(second)/dk (second)^-1 per plane; the 2x2 maps have unit determinant
        const double* M[2] = {a.second.mx, a.second.my};
        const double* D[2] = {a.dfx, a.dfy};
        double* G[2] = {a.dgx, a.dgy};
        for (int p = 0; p < 2; ++p) {
          const double inv[4] = {M[p][3], -M[p][1], -M[p][2], M[p][0]};
          G[p][0] = D[p][0] * inv[0] + D[p][1] * inv[2];
          G[p][1] = D[p][0] * inv[1] + D[p][1] * inv[3];
          G[p][2] = D[p][2] * inv[0] + D[p][3] * inv[2];
          G[p][3] = D[p][2] * inv[1] + D[p][3] * inv[3];
        }
      } else {
        a.dk_kind = kDkNone;
      }
      out.push_back(a);
    }
  }
  return PIC_OK;
}

template <typename T>
pic_status forward_step_recorded(pic_beam b, double* X, const Geom* g, const AdjSlice& e,
                               T* gh, T* E, T* rho, hipStream_t s, Box* box) {
  // the slice's first half map (with the box when a geometry is to be computed), deposit into
  // rho, Green spectrum, solve, kick and the second half map; g is the step's geometry slot
  const int64_t ng = (int64_t)b->d.nx * b->d.ny * b->d.nz;
  HIP_OK(launch_half_box(X, e.first, b->c, box, s), "adjoint forward");
  if (box) HIP_OK(launch_geometry(box, const_cast<Geom*>(g), b->c, s), "adjoint forward");
  HIP_OK(launch_zero<T>(rho, ng, s), "adjoint forward");
  // binned deposit from a tile-sorted copy (XB) of the kick-point state
  HIP_OK(launch_bin(X, b->idA, g, b->c, b->sp, b->keys, b->hist, b->cursor, b->chunks, b->nchunks,
                    b->XB, b->idB, true, s),
         "adjoint forward");
  HIP_OK(launch_deposit_tiles<T>(b->XB, nullptr, g, b->c, b->sp, b->chunks, b->nchunks, rho, s,
                                 b->tacc, b->tscale),
         "adjoint forward");
  if (b->d.direct_field) {  // gh holds the three field kernels' spectra
    HIP_OK(launch_green_field_spectrum<T>(g, b->plan, b->d.nx, b->d.ny, b->d.nz, b->hcorners,
                                          b->gd3, gh, s),
           "adjoint forward");
    HIP_OK(launch_solve_field<T>(g, b->plan, b->d.nx, b->d.ny, b->d.nz, (const T*)rho, b->W,
                                 b->W2, gh, E, s),
           "adjoint forward");
  } else {
    HIP_OK(launch_green_spectrum<T>(g, b->plan, b->d.nx, b->d.ny, b->d.nz, b->corners, b->Gd, gh,
                                    s),
           "adjoint forward");
    HIP_OK(launch_solve<T>(g, b->plan, b->d.nx, b->d.ny, b->d.nz, (const T*)rho, b->W, gh,
                           (T*)b->phi, E, s),
           "adjoint forward");
  }
  HIP_OK(launch_gkd<T>(X, g, E, e.L, e.second, 0, half_drift(0.0), b->c, box, s),
         "adjoint forward");
  return PIC_OK;
}

template <typename T>
pic_status track_adjoint(pic_beam b, const std::vector<AdjSlice>& sl, int n_el, int n_steps,
                         int ck, const double w[4], char* aw, const AdjLayout& A, double* lam,
                         const double* xi, double out_m[4], double* dJ_dk, double dJ_dL[36],
                         hipStream_t s) {
  const size_t nsl = sl.size();
  const bool direct = b->d.direct_field != 0;
  const size_t n = (size_t)b->d.n;
  const int64_t ng = (int64_t)b->d.nx * b->d.ny * b->d.nz;
  // spectra per stored step: the potential's, or the three field kernels'
  const size_t G3 = (size_t)(b->d.nx + 1) * (b->d.ny + 1) * (b->d.nz + 1) *
                    (b->d.direct_field ? 3 : 1);
  auto geom = [&](int j) { return (Geom*)(aw + A.geoms + kGeomSlot * (size_t)j); };
  double* ckpt = (double*)(aw + A.ckpt);
  double* segX = (double*)(aw + A.segX);
  T* segE = (T*)(aw + A.segE);
  T* segG = (T*)(aw + A.segG);
  T* segQ = (T*)(aw + A.segQ);
  T* e = (T*)(aw + A.e);
  T* psi = (T*)(aw + A.psi);
  T* chi = (T*)(aw + A.chi);
  T* chi2 = (T*)(aw + A.chi2);
  double* geo = (double*)(aw + A.geo);
  double* ext_part = (double*)(aw + A.ext_part);
  double* geo_part = (double*)(aw + A.geo_part);
  double* dot_part = (double*)(aw + A.dot_part);
  T* dgh = (T*)(aw + A.dgh);
  const size_t G1 = (size_t)(b->d.nx + 1) * (b->d.ny + 1) * (b->d.nz + 1);
  double* dk = (double*)(aw + A.dk);
  double* small = (double*)(aw + A.small);
  double* P = (double*)(aw + A.stage);
  // the binned vector deposit keeps three float64 windows of a tile in LDS (up to 156 KB)
  const int S = b->d.shape;
  const bool vtiles =
      24 * (size_t)(b->sp.T[0] + S) * (b->sp.T[1] + S) * (b->sp.T[2] + S) <= kMaxLdsBytes;
  HIP_OK(launch_zero<uint32_t>((uint32_t*)(aw + A.geoms), (int64_t)(kGeomSlot / 4) * n_steps, s),
         "adjoint setup");
  HIP_OK(launch_zero<double>(dk, kMaxLattice, s), "adjoint setup");
  // forward: checkpoints at segment starts, geometry of every step kept
  for (int j = 0; j < n_steps; ++j) {
    if (j % ck == 0)
      HIP_OK(hipMemcpyAsync(ckpt + 6 * n * (size_t)(j / ck), b->X, 6 * sizeof(double) * n,
                            hipMemcpyDeviceToDevice, s),
             "adjoint checkpoint");
    HIP_OK(launch_box_reset(b->box, s), "adjoint forward");
    pic_status st = forward_step_recorded<T>(b, b->X, geom(j), sl[j % nsl],
                                           direct ? (T*)b->gh3 : (T*)b->Gh, (T*)b->E,
                                           (T*)b->rho, s, b->box);
    if (st != PIC_OK) return st;
  }
  HIP_OK(launch_moments(b->X, b->d.n, b->mom_partial, b->mom_out, s), "adjoint objective");
  HIP_OK(launch_obj_grad(b->X, b->d.n, b->mom_out, w, lam, small, s), "adjoint objective");
  // reverse, one checkpoint segment at a time
  double* XW = b->XA;
  for (int seg = A.nseg - 1; seg >= 0; --seg) {
    const int c0 = seg * ck, c1 = std::min(c0 + ck, n_steps);
    HIP_OK(hipMemcpyAsync(XW, ckpt + 6 * n * (size_t)seg, 6 * sizeof(double) * n,
                          hipMemcpyDeviceToDevice, s),
           "adjoint recompute");
    for (int j = c0; j < c1; ++j) {
      const int q = j - c0;
      HIP_OK(hipMemcpyAsync(segX + 6 * n * (size_t)q, XW, 6 * sizeof(double) * n,
                            hipMemcpyDeviceToDevice, s),
             "adjoint recompute");
      pic_status st = forward_step_recorded<T>(b, XW, geom(j), sl[j % nsl], segG + G3 * (size_t)q,
                                             segE + 3 * ng * (size_t)q, segQ + ng * (size_t)q, s,
                                             nullptr);
      if (st != PIC_OK) return st;
    }
    for (int j = c1 - 1; j >= c0; --j) {
      const int q = j - c0;
      const AdjSlice& el = sl[j % nsl];
      const double* Xs = segX + 6 * n * (size_t)q;
      // the state after the step: the next stored one, the next segment's checkpoint, or the
      // final state
      const double* Xn = j + 1 < c1 ? segX + 6 * n * (size_t)(q + 1)
                         : j + 1 < n_steps ? ckpt + 6 * n * (size_t)(seg + 1)
                                           : b->X;
      HIP_OK(launch_adj_dk_second(Xn, lam, b->c, el, (double*)(aw + A.dk_part), dk, s),
             "adjoint");
      HIP_OK(launch_zero<T>(e, 3 * ng, s), "adjoint");
      if (vtiles) {
        // kick-point positions and deposit values, tile-sorted, then the binned vector deposit
        HIP_OK(launch_adj_stage(Xs, lam, geom(j), b->c, el, P, ext_part, geo, s), "adjoint");
        HIP_OK(launch_bin(P, b->idA, geom(j), b->c, b->sp, b->keys, b->hist, b->cursor,
                          b->chunks, b->nchunks, b->XB, b->idB, true, s),
               "adjoint");
        HIP_OK(launch_vdeposit_tiles<T>(b->XB, geom(j), b->c, b->sp, b->chunks, b->nchunks, e, s),
               "adjoint");
      } else {
        HIP_OK(launch_adj_a<T>(Xs, lam, geom(j), b->c, el, e, ext_part, geo, s), "adjoint");
      }
      if (direct) {  // transposed field convolutions, b->E as their scratch
        HIP_OK(launch_solve_field_T<T>(geom(j), b->plan, b->d.nx, b->d.ny, b->d.nz, e, b->W, b->W2,
                                       segG + G3 * (size_t)q, (T*)b->E, chi, s),
               "adjoint");
      } else {
        HIP_OK(launch_adj_div<T>(geom(j), e, psi, b->d.nx, b->d.ny, b->d.nz, s), "adjoint");
        HIP_OK(launch_solve_ghost_source<T>(geom(j), b->plan, b->d.nx, b->d.ny, b->d.nz, psi,
                                            b->W, segG + G3 * (size_t)q, chi, s),
               "adjoint");
      }
      HIP_OK(launch_adj_b<T>(Xs, lam, geom(j), b->c, el, segE + 3 * ng * (size_t)q, chi,
                             (double*)(aw + A.dk_part), dk, geo_part, geo, s),
             "adjoint");
      // the geometry's terms: dJ/dh' through the kernel (the h-derivative kernels' convolution
      // with the adjoint source, dotted with the step's charge) into geo[12..14], and through
      // the centred difference sum_n e_b E'_b into geo[15..17] (zero for the direct field)
      const T* Qj = segQ + ng * (size_t)q;
      HIP_OK(launch_green_dh_spectra<T>(geom(j), b->plan, b->d.nx, b->d.ny, b->d.nz, direct,
                                        (double2*)(aw + A.dc), (double*)(aw + A.dgd), dgh, s),
             "adjoint geometry");
      for (int hb = 0; hb < 3; ++hb) {
        if (direct)
          HIP_OK(launch_solve_field_T<T>(geom(j), b->plan, b->d.nx, b->d.ny, b->d.nz, e, b->W,
                                         b->W2, dgh + 3 * G1 * (size_t)hb, (T*)b->E, chi2, s),
                 "adjoint geometry");
        else
          HIP_OK(launch_solve_ghost_source<T>(geom(j), b->plan, b->d.nx, b->d.ny, b->d.nz, psi,
                                              b->W, dgh + G1 * (size_t)hb, chi2, s),
                 "adjoint geometry");
        HIP_OK(launch_grid_dot<T>(Qj, chi2, ng, 1, 0, dot_part, geo + 12 + hb, s),
               "adjoint geometry");
      }
      if (direct)
        HIP_OK(launch_zero<double>(geo + 15, 3, s), "adjoint geometry");
      else
        HIP_OK(launch_grid_dot<T>(e, segE + 3 * ng * (size_t)q, ng, 3, ng, dot_part, geo + 15, s),
               "adjoint geometry");
      HIP_OK(launch_adj_geom(Xs, lam, geom(j), b->c, el, geo, dk, s), "adjoint geometry");
    }
  }
  if (xi)
    HIP_OK(launch_dL(lam, xi, b->d.n, (double*)(aw + A.dL_part), small + 4, s), "adjoint dL");
  // results and the error flags of every step
  double host_small[40];
  HIP_OK(hipMemcpyAsync(host_small, small, sizeof(host_small), hipMemcpyDeviceToHost, s),
         "adjoint results");
  HIP_OK(hipMemcpyAsync(dJ_dk, dk, sizeof(double) * n_el, hipMemcpyDeviceToHost, s),
         "adjoint results");
  std::vector<unsigned char> gbuf(kGeomSlot * (size_t)n_steps);
  HIP_OK(hipMemcpyAsync(gbuf.data(), aw + A.geoms, gbuf.size(), hipMemcpyDeviceToHost, s),
         "adjoint results");
  HIP_OK(hipStreamSynchronize(s), "adjoint results");
  for (int q = 0; q < 4; ++q) out_m[q] = host_small[q];
  if (xi && dJ_dL)
    for (int q = 0; q < 36; ++q) dJ_dL[q] = host_small[4 + q];
  for (int j = 0; j < n_steps; ++j) {
    const Geom* gj = (const Geom*)(gbuf.data() + kGeomSlot * (size_t)j);
    if (gj->status) return device_status(gj->status);
  }
  return PIC_OK;
}

// ---- batches of beams tracked by one graph launch
template <typename T>
pic_status enqueue_batch(const BeamDev* tab, int nb, const BatchDims& bd, int shape, int n_steps,
                         hipStream_t s, hipStream_t aux, hipEvent_t fork, hipEvent_t join) {
  HIP_OK(launch_batch_box_reset(tab, nb, s), "batch");
  HIP_OK(launch_batch_clear_tacc(tab, nb, s), "batch");
  HIP_OK(launch_batch_prologue_particles(tab, nb, bd, s), "batch");
  for (int j = 0; j < n_steps; ++j) {
    const int parity = j & 1;
    HIP_OK(launch_batch_geometry(tab, nb, s), "batch");
    HIP_OK(launch_batch_zero_rho<T>(tab, nb, bd, s), "batch");
    // Green spectra on the auxiliary stream, concurrently with binning and deposit
    HIP_OK(hipEventRecord(fork, s), "batch");
    HIP_OK(hipStreamWaitEvent(aux, fork, 0), "batch");
    HIP_OK(launch_batch_green<T>(tab, nb, bd, aux), "batch");
    HIP_OK(hipEventRecord(join, aux), "batch");
    HIP_OK(launch_batch_particles_bin(tab, nb, bd, shape, parity, j == 0, s), "batch");
    HIP_OK(launch_batch_deposit<T>(tab, nb, bd, shape, parity, j == 0, s), "batch");
    HIP_OK(hipStreamWaitEvent(s, join, 0), "batch");
    HIP_OK(launch_batch_solve<T>(tab, nb, bd, s), "batch");
    if (j + 1 < n_steps) HIP_OK(launch_batch_box_reset(tab, nb, s), "batch");
    HIP_OK(launch_batch_gkd<T>(tab, nb, bd, shape, parity, j, n_steps, j == 0, s), "batch");
  }
  HIP_OK(launch_batch_unpermute(tab, nb, bd, n_steps & 1, s), "batch");
  return PIC_OK;
}

}  // namespace

struct pic_batch_s {
  int nb = 0;
  int shape = 1;
  int fp32 = 0;
  std::vector<pic_beam> beams;
  BeamDev* table = nullptr;  // device, in the caller's batch workspace
  BatchDims bd;
  struct Graph {
    int n_steps;
    hipGraphExec_t exec;
    DoneEvent done;  // recorded after every launch of this graph, on the launch's stream
  };
  std::vector<Graph> graphs;  // one instantiated graph per step count
  hipStream_t aux = nullptr;  // Green spectra, forked from the captured stream
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  ~pic_batch_s() {
    // a graph executable must not be destroyed while a launch of it may still run
    for (auto& g : graphs) g.done.wait();
    if (aux) (void)hipStreamSynchronize(aux);
    for (auto& g : graphs) {
      (void)hipGraphExecDestroy(g.exec);
      if (g.done.ev) (void)hipEventDestroy(g.done.ev);
    }
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (aux) (void)hipStreamDestroy(aux);
  }
};

extern "C" {

const char* pic_last_error(void) { return g_last_error.c_str(); }

size_t pic_workspace_bytes(const pic_beam_desc* d) {
  if (check_desc(d) != PIC_OK) return 0;
  return layout(d).total;
}

pic_status pic_beam_create(const pic_beam_desc* d, double* d_X, void* d_work, size_t work_bytes,
                           void* stream, pic_beam* out) {
  if (!out) return fail(PIC_EINVAL, "NULL output handle");
  *out = nullptr;
  pic_status st = check_desc(d);
  if (st != PIC_OK) return st;
  if (!d_X || !d_work) return fail(PIC_EINVAL, "NULL device pointer");
  if (((uintptr_t)d_X & 7) || ((uintptr_t)d_work & 255))
    return fail(PIC_EINVAL, "X must be 8-byte and the workspace 256-byte aligned");
  Layout L = layout(d);
  if (work_bytes < L.total) return fail(PIC_ENOMEM, "workspace smaller than pic_workspace_bytes");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(PIC_ENODEV, "no HIP device");

  pic_beam b = new (std::nothrow) pic_beam_s;
  if (!b) return fail(PIC_EINVAL, "host allocation of the handle failed");
  b->d = *d;
  b->X = d_X;
  b->work = (char*)d_work;
  b->L = L;
  const double t = d->kin_energy_MeV / d->mass_MeV;
  const double gamma = 1.0 + t;
  const double gb2 = t * (2.0 + t);
  b->c.n = d->n;
  b->c.nx = d->nx;
  b->c.ny = d->ny;
  b->c.nz = d->nz;
  b->c.shape = d->shape;
  b->c.gamma = gamma;
  b->c.inv_gamma2 = 1.0 / (gamma * gamma);
  b->c.C = d->qm_qeeV / gb2;
  b->c.q_macro = std::copysign(d->charge_C, d->qm_qeeV) / (double)d->n;
  char* w = b->work;
  b->geom = (Geom*)(w + L.geom);
  b->box = (Box*)(w + L.box);
  b->mom_partial = (double*)(w + L.mom_partial);
  b->mom_out = (double*)(w + L.mom_out);
  b->corners = (double2*)(w + L.corners);
  b->W = w + L.W;
  b->Gd = (double*)(w + L.Gd);
  b->Gh = w + L.Gh;
  b->rho = w + L.rho;
  b->phi = w + L.phi;
  b->E = w + L.E;
  b->hcorners = (double2*)(w + L.hcorners);
  b->gd3 = (double*)(w + L.gd3);
  b->gh3 = w + L.gh3;
  b->W2 = w + L.W2;
  b->sp = make_sort_plan(d->nx, d->ny, d->nz, d->n, d->tile, d->chunk, d->blocks, d->threads,
                         d->deposit_threads);
  b->XA = (double*)(w + L.XA);
  b->XB = (double*)(w + L.XB);
  b->idA = (uint32_t*)(w + L.idA);
  b->idB = (uint32_t*)(w + L.idB);
  b->keys = (uint32_t*)(w + L.keys);
  b->perm = (uint32_t*)(w + L.perm);
  b->hist = (uint32_t*)(w + L.hist);
  b->cursor = (uint32_t*)(w + L.cursor);
  b->chunks = (int4*)(w + L.chunks);
  b->nchunks = (uint32_t*)(w + L.nchunks);
  b->diag_part = (double*)(w + L.diag_part);
  b->diag_shift = (double*)(w + L.diag_shift);
  b->tacc = (unsigned long long*)(w + L.tacc);
  b->tscale = (int*)(w + L.tscale);
  int nn[3] = {d->nx, d->ny, d->nz};
  for (int a = 0; a < 3; ++a) {
    b->plan.full[a].M = 2 * nn[a];
    b->plan.full[a].nrad = factor(2 * nn[a], b->plan.full[a].rad);
    b->plan.tw[a] = (const double2*)(w + L.tw[a]);
    b->plan.twf[a] = (const float2*)(w + L.twf[a]);
  }
  b->plan.half_x.M = nn[0];
  b->plan.half_x.nrad = factor(nn[0], b->plan.half_x.rad);
  hipStream_t s = S(stream);
  hipError_t e = hipSuccess;
  for (int a = 0; a < 3 && e == hipSuccess; ++a)
    e = launch_twiddles((double2*)b->plan.tw[a], (float2*)b->plan.twf[a], b->plan.full[a].M, s);
  if (e == hipSuccess) e = launch_box_reset(b->box, s);
  if (e == hipSuccess) e = launch_zero<uint32_t>(b->hist, kMaxTiles, s);
  if (e == hipSuccess) e = launch_clear_status(b->geom, s);
  if (e == hipSuccess) e = make_aux(&b->aux, &b->ev_fork, &b->ev_join, &b->done.ev);
  if (e != hipSuccess) {
    if (b->done.ev == nullptr) (void)hipStreamSynchronize(s);  // the set-up kernels above
    delete b;
    return fail_hip(e, "beam set-up");
  }
  b->done.mark(s);
  *out = b;
  return PIC_OK;
}

pic_status pic_beam_destroy(pic_beam b) {
  delete b;
  return PIC_OK;
}

pic_status pic_init_beam(pic_beam b, const double sigma[36], uint64_t seed, double halo_frac,
                         void* stream) {
  if (!b || !sigma) return fail(PIC_EINVAL, "NULL argument");
  MarkDone md{b->done, S(stream)};
  if (!(halo_frac >= 0.0 && halo_frac <= 1.0)) return fail(PIC_EINVAL, "halo_frac must be in [0, 1]");
  Chol L;
  if (!cholesky6(sigma, L)) return fail(PIC_EINVAL, "sigma is not symmetric positive definite");
  int64_t n_halo = (int64_t)std::floor(halo_frac * (double)b->d.n + 0.5);
  hipStream_t s = S(stream);
  HIP_OK(launch_init_philox(b->X, b->d.n, n_halo, seed, L, 0, s), "init_beam");
  HIP_OK(launch_clear_status(b->geom, s), "init_beam");
  b->x_binned = false;
  return PIC_OK;
}

pic_status pic_init_beam_waterbag(pic_beam b, const double sigma[36], uint64_t seed,
                                  void* stream) {
  if (!b || !sigma) return fail(PIC_EINVAL, "NULL argument");
  MarkDone md{b->done, S(stream)};
  Chol L;
  if (!cholesky6(sigma, L)) return fail(PIC_EINVAL, "sigma is not symmetric positive definite");
  hipStream_t s = S(stream);
  HIP_OK(launch_init_philox(b->X, b->d.n, 0, seed, L, 1, s), "init_beam_waterbag");
  HIP_OK(launch_clear_status(b->geom, s), "init_beam_waterbag");
  b->x_binned = false;
  return PIC_OK;
}

pic_status pic_sigma_from_params(const double p[9], double sigma[36]) {
  if (!p || !sigma) return fail(PIC_EINVAL, "NULL argument");
  double S[36] = {0};
  for (int a = 0; a < 3; ++a) {
    const double su = p[a], sp = p[3 + a], mu = p[6 + a];
    if (!(su > 0.0) || !(sp > 0.0) || !std::isfinite(su) || !std::isfinite(sp) ||
        !(std::fabs(mu) < 1.0))
      return fail(PIC_EINVAL, "sigmas must be finite and positive, |mu| < 1");
    const double c = 1.0 / std::sqrt(1.0 - mu * mu);
    const double ru = su * c, rp = sp * c;
    const int i = 2 * a;
    S[i * 6 + i] = ru * ru;
    S[(i + 1) * 6 + i + 1] = rp * rp;
    S[i * 6 + i + 1] = S[(i + 1) * 6 + i] = -mu * ru * rp;
  }
  std::memcpy(sigma, S, sizeof(S));
  return PIC_OK;
}

pic_status pic_init_beam_from_normals(pic_beam b, const double sigma[36], const double* d_xi,
                                      void* stream) {
  if (!b || !sigma || !d_xi) return fail(PIC_EINVAL, "NULL argument");
  if ((uintptr_t)d_xi & 7) return fail(PIC_EINVAL, "xi must be 8-byte aligned");
  MarkDone md{b->done, S(stream)};
  Chol L;
  if (!cholesky6(sigma, L)) return fail(PIC_EINVAL, "sigma is not symmetric positive definite");
  hipStream_t s = S(stream);
  HIP_OK(launch_init_normals(b->X, d_xi, b->d.n, L, s), "init_beam_from_normals");
  HIP_OK(launch_clear_status(b->geom, s), "init_beam_from_normals");
  b->x_binned = false;
  return PIC_OK;
}

namespace {
// a grid or particle-field array must be aligned to its element (pic_real)
bool grid_misaligned(const pic_beam b, const void* p) {
  return p && ((uintptr_t)p & (b->d.grid_fp32 ? 3u : 7u));
}
}  // namespace

pic_status pic_deposit(pic_beam b, void* d_rho, void* stream) {
  if (!b || !d_rho) return fail(PIC_EINVAL, "NULL argument");
  if (grid_misaligned(b, d_rho)) return fail(PIC_EINVAL, "rho must be aligned to its element");
  MarkDone md{b->done, S(stream)};
  hipStream_t s = S(stream);
  const int64_t ng = (int64_t)b->d.nx * b->d.ny * b->d.nz;
  HIP_OK(launch_box_reset(b->box, s), "deposit");
  HIP_OK(launch_box(b->X, b->d.n, b->box, s), "deposit");
  HIP_OK(launch_geometry(b->box, b->geom, b->c, s), "deposit");
  // binned as in the tracking loop: tile keys and the ranking of X (X itself is not moved),
  // then the tiles' integer windows, so the grid does not depend on the order of the atomics
  HIP_OK(clear_tacc(b, s), "deposit");
  HIP_OK(launch_bin_perm(b->X, b->geom, b->c, b->sp, b->keys, b->hist, b->cursor, b->chunks,
                         b->nchunks, b->perm, s),
         "deposit");
  if (b->d.grid_fp32) {
    HIP_OK(launch_zero<float>((float*)d_rho, ng, s), "deposit");
    HIP_OK(launch_deposit_tiles<float>(b->X, b->perm, b->geom, b->c, b->sp, b->chunks,
                                       b->nchunks, (float*)d_rho, s, b->tacc, b->tscale),
           "deposit");
  } else {
    HIP_OK(launch_zero<double>((double*)d_rho, ng, s), "deposit");
    HIP_OK(launch_deposit_tiles<double>(b->X, b->perm, b->geom, b->c, b->sp, b->chunks,
                                        b->nchunks, (double*)d_rho, s, b->tacc, b->tscale),
           "deposit");
  }
  return PIC_OK;
}

pic_status pic_poisson_solve(pic_beam b, const void* d_rho, void* d_phi, void* d_E, void* stream) {
  if (!b || !d_rho || !d_E) return fail(PIC_EINVAL, "NULL argument");
  if (grid_misaligned(b, d_rho) || grid_misaligned(b, d_phi) || grid_misaligned(b, d_E))
    return fail(PIC_EINVAL, "rho, phi and E must be aligned to their element");
  MarkDone md{b->done, S(stream)};
  hipStream_t s = S(stream);
  void* phi = d_phi ? d_phi : b->phi;
  if (b->d.direct_field && d_phi) {  // phi as well: the potential's spectrum and solve
    if (b->d.grid_fp32)
      HIP_OK((launch_green_spectrum<float>(b->geom, b->plan, b->d.nx, b->d.ny, b->d.nz,
                                          b->corners, b->Gd, (float*)b->Gh, s)), "poisson solve");
    else
      HIP_OK((launch_green_spectrum<double>(b->geom, b->plan, b->d.nx, b->d.ny, b->d.nz,
                                           b->corners, b->Gd, (double*)b->Gh, s)), "poisson solve");
    if (b->d.grid_fp32)
      HIP_OK(launch_solve<float>(b->geom, b->plan, b->d.nx, b->d.ny, b->d.nz,
                                 (const float*)d_rho, b->W, (const float*)b->Gh, (float*)d_phi,
                                 (float*)b->E, s), "poisson solve");
    else
      HIP_OK(launch_solve<double>(b->geom, b->plan, b->d.nx, b->d.ny, b->d.nz,
                                  (const double*)d_rho, b->W, (const double*)b->Gh,
                                  (double*)d_phi, (double*)b->E, s), "poisson solve");
  }
  if (b->d.grid_fp32)
    return green_and_solve<float>(b, (const float*)d_rho, (float*)phi, (float*)d_E, s);
  return green_and_solve<double>(b, (const double*)d_rho, (double*)phi, (double*)d_E, s);
}

pic_status pic_gather(pic_beam b, const void* d_E, void* d_Ep, void* stream) {
  if (!b || !d_E || !d_Ep) return fail(PIC_EINVAL, "NULL argument");
  if (grid_misaligned(b, d_E) || grid_misaligned(b, d_Ep))
    return fail(PIC_EINVAL, "E and Ep must be aligned to their element");
  MarkDone md{b->done, S(stream)};
  hipStream_t s = S(stream);
  if (b->d.grid_fp32)
    HIP_OK(launch_gather<float>(b->X, b->geom, (const float*)d_E, (float*)d_Ep, b->c, s), "gather");
  else
    HIP_OK(launch_gather<double>(b->X, b->geom, (const double*)d_E, (double*)d_Ep, b->c, s),
           "gather");
  return PIC_OK;
}

pic_status pic_push(pic_beam b, int kind, double value, const void* d_Ep, void* stream) {
  if (!b) return fail(PIC_EINVAL, "NULL handle");
  MarkDone md{b->done, S(stream)};
  if (kind != PIC_PUSH_DRIFT && kind != PIC_PUSH_THINQUAD && kind != PIC_PUSH_KICK)
    return fail(PIC_EINVAL, "unknown push kind");
  if (kind == PIC_PUSH_KICK && !d_Ep) return fail(PIC_EINVAL, "kick needs the particle field");
  if (kind == PIC_PUSH_KICK && grid_misaligned(b, d_Ep))
    return fail(PIC_EINVAL, "Ep must be aligned to its element");
  if (!std::isfinite(value)) return fail(PIC_EINVAL, "non-finite push parameter");
  hipStream_t s = S(stream);
  if (b->d.grid_fp32)
    HIP_OK(launch_push<float>(b->X, kind, value, (const float*)d_Ep, b->c, s), "push");
  else
    HIP_OK(launch_push<double>(b->X, kind, value, (const double*)d_Ep, b->c, s), "push");
  return PIC_OK;
}

namespace {
pic_status track(pic_beam b, const pic_element* lattice, int n_el, int n_steps, double* diag,
                 void* stream, bool binned = false, uint32_t* ids_io = nullptr) {
  if (!b || !lattice) return fail(PIC_EINVAL, "NULL argument");
  MarkDone md{b->done, S(stream)};
  if (n_el < 1 || n_steps < 0) return fail(PIC_EINVAL, "n_el must be >= 1 and n_steps >= 0");
  std::vector<SliceDev> sl;
  const pic_status est = expand_lattice(lattice, n_el, sl);
  if (est != PIC_OK) return est;
  if (n_steps == 0) return PIC_OK;
  hipStream_t s = S(stream);
  if (!b->d.space_charge) {
    for (int j = 0; j < n_steps; ++j) {
      const SliceDev& e = sl[j % sl.size()];
      HIP_OK(launch_half_maps(b->X, e.first, e.second, b->c, s), "track");
      if (diag)
        HIP_OK(launch_moments(b->X, b->d.n, b->mom_partial, diag + (size_t)kMomentSlots * j, s),
               "diagnostics");
    }
    return PIC_OK;
  }
  const bool first_ranked = binned && b->x_binned;
  const pic_status st =
      b->d.grid_fp32 ? track_sc<float>(b, sl, n_steps, diag, s, binned, ids_io, first_ranked)
                     : track_sc<double>(b, sl, n_steps, diag, s, binned, ids_io, first_ranked);
  if (st == PIC_OK && binned) b->x_binned = true;
  return st;
}
}  // namespace

pic_status pic_track_n_steps(pic_beam b, const pic_element* lattice, int n_el, int n_steps,
                             void* stream) {
  return track(b, lattice, n_el, n_steps, nullptr, stream);
}

pic_status pic_track_n_steps_binned(pic_beam b, const pic_element* lattice, int n_el,
                                    int n_steps, uint32_t* d_ids, void* stream) {
  if (d_ids && ((uintptr_t)d_ids & 3)) return fail(PIC_EINVAL, "d_ids must be 4-byte aligned");
  return track(b, lattice, n_el, n_steps, nullptr, stream, true, d_ids);
}

pic_status pic_track_n_steps_diag(pic_beam b, const pic_element* lattice, int n_el, int n_steps,
                                  double* d_diag, void* stream) {
  if (!d_diag) return fail(PIC_EINVAL, "NULL diagnostics array");
  if ((uintptr_t)d_diag & 7) return fail(PIC_EINVAL, "the diagnostics array must be 8-byte aligned");
  return track(b, lattice, n_el, n_steps, d_diag, stream);
}

pic_status pic_moments(pic_beam b, double mean[6], double cov[36], void* stream) {
  if (!b || !mean || !cov) return fail(PIC_EINVAL, "NULL argument");
  MarkDone md{b->done, S(stream)};
  hipStream_t s = S(stream);
  HIP_OK(launch_moments(b->X, b->d.n, b->mom_partial, b->mom_out, s), "moments");
  double host[kMomentSlots];
  Geom g;
  HIP_OK(hipMemcpyAsync(host, b->mom_out, sizeof(host), hipMemcpyDeviceToHost, s), "moments");
  HIP_OK(hipMemcpyAsync(&g, b->geom, sizeof(Geom), hipMemcpyDeviceToHost, s), "moments");
  HIP_OK(hipStreamSynchronize(s), "moments");
  for (int r = 0; r < 6; ++r) mean[r] = host[r];
  int q = 6;
  for (int a = 0; a < 6; ++a)
    for (int c = a; c < 6; ++c) {
      cov[a * 6 + c] = cov[c * 6 + a] = host[q++];
    }
  return device_status(g.status);
}

pic_status pic_objective(pic_beam b, double out_m[4], void* stream) {
  if (!b || !out_m) return fail(PIC_EINVAL, "NULL argument");
  MarkDone md{b->done, S(stream)};
  hipStream_t s = S(stream);
  HIP_OK(launch_moments(b->X, b->d.n, b->mom_partial, b->mom_out, s), "objective");
  HIP_OK(launch_objective(b->mom_out, b->mom_out + kMomentSlots, s), "objective");
  Geom g;
  HIP_OK(hipMemcpyAsync(out_m, b->mom_out + kMomentSlots, 4 * sizeof(double),
                        hipMemcpyDeviceToHost, s),
         "objective");
  HIP_OK(hipMemcpyAsync(&g, b->geom, sizeof(Geom), hipMemcpyDeviceToHost, s), "objective");
  HIP_OK(hipStreamSynchronize(s), "objective");
  return device_status(g.status);
}

pic_status pic_get_geometry(pic_beam b, double out[9], void* stream) {
  if (!b || !out) return fail(PIC_EINVAL, "NULL argument");
  hipStream_t s = S(stream);
  Geom g;
  HIP_OK(hipMemcpyAsync(&g, b->geom, sizeof(Geom), hipMemcpyDeviceToHost, s), "geometry");
  HIP_OK(hipStreamSynchronize(s), "geometry");
  for (int a = 0; a < 3; ++a) {
    out[a] = g.origin[a];
    out[3 + a] = g.h[a];
    out[6 + a] = g.h_rest[a];
  }
  return device_status(g.status);
}

size_t pic_adjoint_workspace_bytes(const pic_beam_desc* d, int n_steps, int ckpt_every) {
  if (check_desc(d) != PIC_OK || n_steps < 1 || ckpt_every < 1) return 0;
  return adj_layout(d, n_steps, ckpt_every).total;
}

pic_status pic_track_adjoint(pic_beam b, const pic_element* lattice, int n_el, int n_steps,
                             int ckpt_every, const double w[4], void* d_adj_work,
                             size_t adj_work_bytes, double* d_lam, const double* d_xi,
                             double out_m[4], double* dJ_dk, double dJ_dL[36], void* stream) {
  if (!b || !lattice || !w || !d_adj_work || !d_lam || !out_m || !dJ_dk)
    return fail(PIC_EINVAL, "NULL argument");
  if (n_el < 1 || n_el > kMaxLattice || n_steps < 1 || ckpt_every < 1)
    return fail(PIC_EINVAL, "need 1 <= n_el <= 1024, n_steps >= 1, ckpt_every >= 1");
  if (!b->d.space_charge) return fail(PIC_EINVAL, "the reverse sweep needs space_charge = 1");
  if (d_xi && !dJ_dL) return fail(PIC_EINVAL, "d_xi given without dJ_dL");
  if ((uintptr_t)d_adj_work & 255) return fail(PIC_EINVAL, "workspace must be 256-byte aligned");
  if (((uintptr_t)d_lam & 7) || ((uintptr_t)d_xi & 7))
    return fail(PIC_EINVAL, "lam and xi must be 8-byte aligned");
  std::vector<AdjSlice> sl;
  const pic_status est = expand_adjoint(lattice, n_el, sl);
  if (est != PIC_OK) return est;
  for (int q = 0; q < 4; ++q)
    if (!std::isfinite(w[q])) return fail(PIC_EINVAL, "non-finite objective weight");
  AdjLayout A = adj_layout(&b->d, n_steps, ckpt_every);
  if (adj_work_bytes < A.total)
    return fail(PIC_ENOMEM, "reverse-sweep workspace smaller than pic_adjoint_workspace_bytes");
  hipStream_t s = S(stream);
  MarkDone md{b->done, s};
  HIP_OK(clear_tacc(b, s), "clear");
  if (b->d.grid_fp32)
    return track_adjoint<float>(b, sl, n_el, n_steps, ckpt_every, w, (char*)d_adj_work, A,
                                d_lam, d_xi, out_m, dJ_dk, dJ_dL, s);
  return track_adjoint<double>(b, sl, n_el, n_steps, ckpt_every, w, (char*)d_adj_work, A,
                               d_lam, d_xi, out_m, dJ_dk, dJ_dL, s);
}

size_t pic_batch_workspace_bytes(int n_beams, const pic_element* const* lattices,
                                 const int* n_el) {
  if (n_beams < 1 || !n_el || !lattices) return 0;
  size_t nsl = 0;
  std::vector<SliceDev> sl;
  for (int b = 0; b < n_beams; ++b) {
    if (n_el[b] < 1 || !lattices[b]) return 0;
    if (expand_lattice(lattices[b], n_el[b], sl) != PIC_OK) return 0;
    nsl += sl.size();
  }
  return align256(sizeof(BeamDev) * (size_t)n_beams) + align256(sizeof(SliceDev) * nsl);
}

pic_status pic_batch_create(pic_beam* beams, int n_beams, const pic_element* const* lattices,
                            const int* n_el, int blocks_per_beam, void* d_work,
                            size_t work_bytes, void* stream, pic_batch* out) {
  if (!out) return fail(PIC_EINVAL, "NULL output handle");
  *out = nullptr;
  if (!beams || !lattices || !n_el || !d_work || n_beams < 1)
    return fail(PIC_EINVAL, "NULL argument or no beams");
  if ((uintptr_t)d_work & 255) return fail(PIC_EINVAL, "workspace must be 256-byte aligned");
  if (blocks_per_beam < 0 || blocks_per_beam > 65535)
    return fail(PIC_EINVAL, "blocks_per_beam must be 0..65535");
  const size_t need = pic_batch_workspace_bytes(n_beams, lattices, n_el);
  if (need == 0) return fail(PIC_EINVAL, "every beam needs a lattice of >= 1 element");
  if (work_bytes < need) return fail(PIC_ENOMEM, "batch workspace smaller than pic_batch_workspace_bytes");
  const int shape = beams[0] ? beams[0]->d.shape : 0;
  const int fp32 = beams[0] ? beams[0]->d.grid_fp32 : 0;
  BatchDims bd{};
  std::vector<BeamDev> tab(n_beams);
  std::vector<SliceDev> all, sl;
  std::vector<size_t> lat_off(n_beams);
  for (int b = 0; b < n_beams; ++b) {
    pic_beam h = beams[b];
    if (!h || !lattices[b]) return fail(PIC_EINVAL, "NULL beam or lattice");
    if (h->d.shape != shape || h->d.grid_fp32 != fp32 || !h->d.space_charge)
      return fail(PIC_EINVAL, "beams of a batch share shape and grid precision and need space charge");
    if (h->d.direct_field)
      return fail(PIC_EUNSUPPORTED, "batched beams use the differenced field");
    const size_t es = fp32 ? 4 : 8;
    const size_t nodes = (size_t)(h->sp.T[0] + shape) * (h->sp.T[1] + shape) * (h->sp.T[2] + shape);
    const size_t win = es * nodes;
    if (3 * win > kMaxLdsBytes)
      return fail(PIC_EUNSUPPORTED, "tile window of a batched beam exceeds 156 KB");
    bd.max_n = std::max<int64_t>(bd.max_n, h->d.n);
    bd.max_nx = std::max(bd.max_nx, h->d.nx);
    bd.max_ny = std::max(bd.max_ny, h->d.ny);
    bd.max_nz = std::max(bd.max_nz, h->d.nz);
    bd.dep_lds = std::max(bd.dep_lds, sizeof(unsigned long long) * nodes);
    bd.gkd_lds = std::max(bd.gkd_lds, 3 * win);
    lat_off[b] = all.size();
    const pic_status est = expand_lattice(lattices[b], n_el[b], sl);
    if (est != PIC_OK) return est;
    all.insert(all.end(), sl.begin(), sl.end());
    BeamDev& d = tab[b];
    d.c = h->c;
    d.sp = h->sp;
    d.plan = h->plan;
    d.X = h->X;
    d.XA = h->XA;
    d.XB = h->XB;
    d.idA = h->idA;
    d.idB = h->idB;
    d.keys = h->keys;
    d.perm = h->perm;
    d.hist = h->hist;
    d.cursor = h->cursor;
    d.chunks = h->chunks;
    d.nchunks = h->nchunks;
    d.geom = h->geom;
    d.box = h->box;
    d.rho = h->rho;
    d.phi = h->phi;
    d.E = h->E;
    d.W = h->W;
    d.Gd = h->Gd;
    d.Gh = h->Gh;
    d.corners = h->corners;
    d.tacc = h->tacc;
    d.tscale = h->tscale;
    d.n_slices = (int)sl.size();
  }
  // per-beam work-list blocks of the tiled kernels: the blocks of a beam stride over its chunks
  bd.max_chunks = blocks_per_beam > 0 ? blocks_per_beam : 256;
  char* w = (char*)d_work;
  BeamDev* dtab = (BeamDev*)w;
  SliceDev* dlat = (SliceDev*)(w + align256(sizeof(BeamDev) * (size_t)n_beams));
  for (int b = 0; b < n_beams; ++b) tab[b].slices = dlat + lat_off[b];
  hipStream_t s = S(stream);
  HIP_OK(hipMemcpyAsync(dtab, tab.data(), sizeof(BeamDev) * tab.size(), hipMemcpyHostToDevice, s),
         "batch create");
  HIP_OK(hipMemcpyAsync(dlat, all.data(), sizeof(SliceDev) * all.size(), hipMemcpyHostToDevice,
                        s),
         "batch create");
  HIP_OK(hipStreamSynchronize(s), "batch create");
  pic_batch bt = new (std::nothrow) pic_batch_s;
  if (!bt) return fail(PIC_EINVAL, "host allocation of the batch handle failed");
  hipEvent_t unused_done = nullptr;
  const hipError_t ea = make_aux(&bt->aux, &bt->ev_fork, &bt->ev_join, &unused_done);
  if (unused_done) (void)hipEventDestroy(unused_done);  // a batch keeps one per graph instead
  if (ea != hipSuccess) {
    delete bt;
    return fail_hip(ea, "batch create");
  }
  bt->nb = n_beams;
  bt->shape = shape;
  bt->fp32 = fp32;
  bt->beams.assign(beams, beams + n_beams);
  bt->table = dtab;
  bt->bd = bd;
  *out = bt;
  return PIC_OK;
}

pic_status pic_track_batch(pic_batch bt, int n_steps, void* stream) {
  if (!bt) return fail(PIC_EINVAL, "NULL batch");
  if (n_steps < 1) return fail(PIC_EINVAL, "n_steps must be >= 1");
  if (!stream) return fail(PIC_EINVAL, "a batch is captured into a graph: pass a non-null stream");
  hipStream_t s = S(stream);
  pic_batch_s::Graph* gr = nullptr;
  for (auto& g : bt->graphs)
    if (g.n_steps == n_steps) gr = &g;
  if (!gr) {
    hipGraphExec_t exec = nullptr;
    HIP_OK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "batch capture");
    pic_status st =
        bt->fp32 ? enqueue_batch<float>(bt->table, bt->nb, bt->bd, bt->shape, n_steps, s, bt->aux,
                                        bt->ev_fork, bt->ev_join)
                 : enqueue_batch<double>(bt->table, bt->nb, bt->bd, bt->shape, n_steps, s,
                                         bt->aux, bt->ev_fork, bt->ev_join);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(s, &graph);
    if (st != PIC_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return st;
    }
    if (e != hipSuccess) return fail_hip(e, "batch capture");
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail_hip(e, "batch graph instantiation");
    hipEvent_t done = nullptr;
    e = hipEventCreateWithFlags(&done, hipEventDisableTiming);
    if (e != hipSuccess) {
      (void)hipGraphExecDestroy(exec);
      return fail_hip(e, "batch graph event");
    }
    bt->graphs.push_back(pic_batch_s::Graph{n_steps, exec, DoneEvent{done, false}});
    gr = &bt->graphs.back();
  }
  HIP_OK(hipGraphLaunch(gr->exec, s), "batch graph launch");
  gr->done.mark(s);
  return PIC_OK;
}

pic_status pic_batch_destroy(pic_batch bt) {
  delete bt;
  return PIC_OK;
}

pic_status pic_profile_start(pic_beam b) {
  if (!b) return fail(PIC_EINVAL, "NULL handle");
  b->prof.on = true;
  b->prof.used = 0;
  return PIC_OK;
}

pic_status pic_profile_read(pic_beam b, double ms[8], int64_t launches[8]) {
  if (!b || !ms || !launches) return fail(PIC_EINVAL, "NULL argument");
  for (int q = 0; q < PIC_NSTAGES; ++q) {
    ms[q] = 0.0;
    launches[q] = 0;
  }
  StageProfiler& p = b->prof;
  for (size_t k = 0; k < p.used; ++k) {
    HIP_OK(hipEventSynchronize(p.pool[2 * k + 1]), "profile read");
    float t = 0.f;
    HIP_OK(hipEventElapsedTime(&t, p.pool[2 * k], p.pool[2 * k + 1]), "profile read");
    ms[p.stage[k]] += (double)t;
    launches[p.stage[k]] += 1;
  }
  p.on = false;
  p.used = 0;
  return PIC_OK;
}

pic_status pic_check(pic_beam b, void* stream) {
  if (!b) return fail(PIC_EINVAL, "NULL handle");
  hipStream_t s = S(stream);
  Geom g;
  HIP_OK(hipMemcpyAsync(&g, b->geom, sizeof(Geom), hipMemcpyDeviceToHost, s), "check");
  HIP_OK(hipStreamSynchronize(s), "check");
  return device_status(g.status);
}

}  // extern "C"
