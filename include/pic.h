/*
 * pic.h -- C ABI of libpic.so, a space-charge particle-in-cell step for s-based beam dynamics
 * on AMD Instinct MI355X (gfx950).
 *
 * The method (arXiv:2208.02382, section "Model Assumptions"): particles are pushed in s by
 * symplectic maps that are linear about the reference orbit; space charge is electrostatic in
 * the bunch rest frame, obtained from a Poisson solve there and applied with a split-operator
 * (kick between two half drifts).  The paper names the building blocks -- charge deposition,
 * Poisson solve, beam statistics (section "ImpactX") -- and the user-level calls of its
 * Listing 1: add_particles(qm, charge_C, distribution, npart), set_particle_shape(order),
 * ref_particle().set_energy_MeV(E, mass), set_space_charge(bool), lattice.extend([...]),
 * evolve().  The calls below follow that statement of the problem.
 *
 * Conventions shared by every call
 * --------------------------------
 * Phase space: caller-owned device array X of 6*n doubles, structure of arrays, rows
 *   X[0*n+i] = x [m], X[1*n+i] = px = p_x/p0, X[2*n+i] = y [m], X[3*n+i] = py,
 *   X[4*n+i] = z [m] (lab offset from the reference particle, head positive),
 *   X[5*n+i] = delta = (p - p0)/p0.
 * Grids: node-centred, nx*ny*nz nodes, index ((k*ny)+j)*nx+i (x fastest).  Element type is
 *   double, or float when pic_beam_desc.grid_fp32 = 1 ("pic_real" below).
 * Geometry: each pic_deposit / pic_track_n_steps step takes the box of the particle positions
 *   (min/max of x, y, z); h_a = (max_a - min_a)/(n_a - 3.5), node 0 at min_a - 1.25 h_a, so
 *   every CIC and TSC stencil stays on nodes 0..n_a-1 and the extreme particles sit a quarter
 *   cell from any node or cell boundary.  The rest-frame cell is (hx, hy, gamma*hz).
 * Memory: the library never allocates device memory.  The caller owns X, every grid and the
 *   workspace (size from pic_workspace_bytes).  Workspaces are 256-byte aligned; X, grids and
 *   the other arrays are aligned to their element (8 bytes for double, 4 for float and the
 *   uint32 labels); a misaligned pointer is PIC_EINVAL.  The handle (host memory) is owned by
 *   the library until pic_beam_destroy.
 * Streams: every call takes a hipStream_t as `void* stream` (NULL = the null stream) and only
 *   enqueues work on it, unless stated "synchronises".
 * Errors: calls return pic_status.  Argument errors are reported synchronously and leave the
 *   device untouched.  Device-side errors (a non-finite coordinate, a zero-extent box) set a
 *   flag in the workspace; from then on every kernel of the beam skips its work, and the next
 *   synchronising call (pic_check, pic_moments, pic_get_geometry) returns PIC_EDOMAIN (or
 *   PIC_EINTERNAL for a fault of the library itself).
 *   pic_last_error() gives a message for the last failure on the calling thread.
 * Thread safety: one handle must not be used from two host threads at once; calls on one
 *   handle on two streams race.
 */
#ifndef PIC_H
#define PIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PIC_OK = 0,
  PIC_EINVAL = -1,        /* bad argument (NULL pointer, size, unsupported combination) */
  PIC_ENOMEM = -2,        /* workspace too small */
  PIC_EHIP = -3,          /* a HIP runtime call failed */
  PIC_EDOMAIN = -4,       /* device flagged a non-finite coordinate or a zero-extent box */
  PIC_EUNSUPPORTED = -5,  /* unsupported size or combination: a padded FFT length not 2^a 3^b
                             or > 512, n >= 2^31, the direct field or an oversized tile window
                             in a batch */
  PIC_ENODEV = -6,        /* no HIP device */
  PIC_EINTERNAL = -7      /* the device detected an inconsistency of the library's own binning */
} pic_status;

/* Beam description; mirrors add_particles + set_energy_MeV + set_particle_shape +
 * set_space_charge of the paper's Listing 1. */
typedef struct {
  int64_t n;               /* number of macroparticles (npart), 1 <= n < 2^31 */
  double qm_qeeV;          /* species charge/mass in e/eV (electron: -1e-6/0.510998950) */
  double charge_C;         /* bunch charge magnitude in coulomb; macro charge = sign(qm)*charge_C/n */
  double kin_energy_MeV;   /* reference particle kinetic energy; gamma = 1 + T/m */
  double mass_MeV;         /* rest mass */
  int shape;               /* B-spline order: 1 = CIC, 2 = TSC */
  int nx, ny, nz;          /* grid nodes per axis, each >= 4; padded FFT length 2*n_a must be
                              2^a 3^b and <= 512 */
  int grid_fp32;           /* 0: float64 charge grid, FFT and field; 1: float32 (particles and
                              the push stay float64) */
  int space_charge;        /* 0/1 (set_space_charge); 0 makes pic_track_n_steps purely linear */
  /* Launch tuning of the binned deposit and gather (0 = the library's default for each).
   * pic_track_n_steps gives the same bits for every chunk, blocks, threads and
   * deposit_threads; the tile shape
   * changes only the rounding of the deposit's fixed-point charges (below 1e-13 of a
   * macroparticle's charge per contribution). */
  int tile[3];             /* tile edge in nodes per axis for the per-step binning; the tile
                              count prod(ceil(n_a/tile_a)) must be <= 4096 and the charge
                              window 8 prod(tile_a + shape) bytes <= 156 KB (the dynamic LDS
                              of one workgroup); a field window 3 prod(tile_a + shape) grid
                              elements above 156 KB makes the gather fall back to global
                              loads; default
                              max(4, ceil(n_a/16)) */
  int chunk;               /* max particles per work item of a tile, 256..2^20; default 8192 */
  int blocks;              /* workgroups of the binned deposit and gather, 1..65535; default
                              min(work items, 4096) */
  int threads;             /* threads per workgroup of the binned deposit and gather: a
                              multiple of 64 in 64..1024; default 256 */
  int direct_field;        /* 0: E' = -grad phi by centred differences of the integrated-Green's-
                              function potential; 1: E' from the integrated Green's functions
                              of the field itself (the cell averages of u_a/|r|^3; no
                              differencing error), three convolutions instead of one.  1 is not
                              supported in batches (PIC_EUNSUPPORTED) */
  int deposit_threads;     /* launch tuning: threads per workgroup of the binned charge deposit
                              alone, a multiple of 64 in 64..1024; default (0) that of
                              `threads` */
} pic_beam_desc;

/* Lattice element kinds (Listing 1 of the paper: Drift(ds, nslice), Quad(ds, k, nslice)).
 * pic_track_n_steps takes one step per slice, cycling over the expanded slice list; each step
 * is the split-operator step: the slice's first half map, the space-charge kick over the
 * slice length, the second half map.
 *   PIC_ELEM_THIN   one step: thin quadrupole of integrated strength k [1/m] (px -= k x,
 *                   py += k y), drift ds/2, kick over ds, drift ds/2 (nslice is ignored)
 *   PIC_ELEM_DRIFT  nslice steps of length ds/nslice: drift, kick, drift (k is ignored)
 *   PIC_ELEM_QUAD   nslice steps of length l = ds/nslice of a quadrupole of strength k
 *                   [1/m^2], focusing in x for k > 0: (x, px) <- [[cos p, sin p/sqrt k],
 *                   [-sqrt k sin p, cos p]] (x, px), p = sqrt(k) l/2, cosh/sinh in y; z drifts
 * A zero-initialised element is PIC_ELEM_THIN. */
enum { PIC_ELEM_THIN = 0, PIC_ELEM_DRIFT = 1, PIC_ELEM_QUAD = 2 };
typedef struct {
  double k;     /* strength: [1/m] for PIC_ELEM_THIN, [1/m^2] for PIC_ELEM_QUAD */
  double ds;    /* length [m], >= 0 */
  int kind;     /* PIC_ELEM_* */
  int nslice;   /* slices of a DRIFT or QUAD element, 1..1e6 */
} pic_element;

typedef struct pic_beam_s* pic_beam;
typedef struct pic_batch_s* pic_batch;

/* Push kinds of pic_push. */
enum { PIC_PUSH_DRIFT = 0, PIC_PUSH_THINQUAD = 1, PIC_PUSH_KICK = 2 };

/* Workspace bytes needed for a beam described by d (0 on an invalid description). */
size_t pic_workspace_bytes(const pic_beam_desc* d);

/* Bind a description, the caller's phase-space array d_X (6*n doubles) and workspace to a new
 * handle; enqueues a one-time set-up of the workspace (FFT twiddles, box slots) on `stream`.
 * PIC_ENOMEM if work_bytes < pic_workspace_bytes(d). */
pic_status pic_beam_create(const pic_beam_desc* d, double* d_X, void* d_work, size_t work_bytes,
                           void* stream, pic_beam* out);

/* Release the handle (host memory only; device memory stays the caller's). */
pic_status pic_beam_destroy(pic_beam b);

/* init_beam: fill X with x = L xi, L the lower Cholesky factor of sigma6x6 (row-major 6x6,
 * symmetric positive definite; PIC_EINVAL otherwise).  xi is drawn on the device with
 * Philox4x32-10 (Salmon et al., SC'11; key = seed, counter = (particle index, draw block)) and
 * Box-Muller; the trailing round(halo_frac*n) particles are instead uniform in [-4, 4]^6
 * (a uniform halo out to 4 sigma).  halo_frac in [0, 1]. */
pic_status pic_init_beam(pic_beam b, const double sigma6x6[36], uint64_t seed, double halo_frac,
                         void* stream);

/* Waterbag beam (Listing 1: distribution.Waterbag): X uniform inside the 6-D ellipsoid
 * x^T sigma^-1 x <= 8, whose covariance is sigma6x6 (row-major, symmetric positive definite;
 * PIC_EINVAL otherwise).  x = L xi with xi uniform in the ball of radius sqrt(8): the direction
 * of the six Box-Muller normals of pic_init_beam's draw blocks 0-2 (no halo), times
 * sqrt(8) u^(1/6) with u the first uniform of draw block 3 of the same Philox4x32-10 stream. */
pic_status pic_init_beam_waterbag(pic_beam b, const double sigma6x6[36], uint64_t seed,
                                  void* stream);

/* Covariance (x, px, y, py, z, delta) from the distribution parameters of Listing 1, in the
 * order p = {sigmaX, sigmaY, sigmaT, sigmaPx, sigmaPy, sigmaPt, muxpx, muypy, mutpt}: in each
 * plane the rms size is sigmaU/sqrt(1 - mu^2), the rms momentum sigmaPu/sqrt(1 - mu^2) and the
 * correlation coefficient -mu; (t, pt) are taken as (z, delta).  Host only (no device, no
 * stream).  PIC_EINVAL unless every sigma is finite and positive and |mu| < 1. */
pic_status pic_sigma_from_params(const double params[9], double sigma6x6[36]);

/* Same as pic_init_beam with caller-supplied draws: d_xi is a device array of 6*n doubles in
 * the layout of X.  Used to start the device and a reference implementation from the same
 * draws. */
pic_status pic_init_beam_from_normals(pic_beam b, const double sigma6x6[36], const double* d_xi,
                                      void* stream);

/* Charge deposition (paper: "charge deposition"; shape order of Listing 1): computes the
 * geometry from the current positions, then writes the charge per node in coulomb,
 * Q_n = sum_i q_macro W(x_i - X_n) with W the CIC or TSC tensor-product B-spline, into
 * d_rho (nx*ny*nz pic_real, overwritten).  Binned as in pic_track_n_steps (tile keys and
 * ranking in the workspace; X is not modified) and bitwise reproducible. */
pic_status pic_deposit(pic_beam b, void* d_rho, void* stream);

/* Poisson solve in the bunch rest frame (paper: "Poisson solve"; section "Model Assumptions"):
 * phi_n = 1/(4 pi eps0) sum_m Q_m Gbar(n - m), Gbar the integrated Green's function (cell
 * average of 1/r over a rest-frame cell; Qiang et al., PRST-AB 9, 044204, 2006), by zero
 * padding to (2nz, 2ny, 2nx) and FFT convolution; then E' = -grad phi by centred differences
 * with spacings (hx, hy, gamma hz), or, with pic_beam_desc.direct_field, E'_a = 1/(4 pi eps0)
 * sum_m Q_m Kbar_a(n - m) with Kbar_a the cell average of u_a/|r|^3 (the exact field of the
 * cell-uniform charge; phi is then computed only when d_phi is given).  Uses the geometry of
 * the last pic_deposit.
 * d_rho: nx*ny*nz pic_real (coulomb per node).  d_phi: optional (NULL allowed),
 * (nx+2)*(ny+2)*(nz+2) pic_real holding phi on nodes -1..n_a (volt).  d_E: 3*nx*ny*nz
 * pic_real, component-major E'[c][k][j][i] (V/m, rest frame). */
pic_status pic_poisson_solve(pic_beam b, const void* d_rho, void* d_phi, void* d_E, void* stream);

/* Field gather with the deposit's shape (momentum-conserving): d_Ep[c*n+i] = sum_n
 * W(x_i - X_n) E'[c][n]; d_E as written by pic_poisson_solve, d_Ep 3*n pic_real.
 * Uses the geometry of the last pic_deposit. */
pic_status pic_gather(pic_beam b, const void* d_E, void* d_Ep, void* stream);

/* One linear map on every particle (section "Model Assumptions": maps linear about the
 * reference orbit):
 *   PIC_PUSH_DRIFT     value = l  : x += l px, y += l py, z += l delta/gamma^2
 *   PIC_PUSH_THINQUAD  value = k  : px -= k x, py += k y
 *   PIC_PUSH_KICK      value = L  : px += C E'x L, py += C E'y L, delta += gamma C E'z L with
 *                                   C = qm_qeeV/(gamma^2 beta^2) and d_Ep from pic_gather
 * d_Ep is read only by PIC_PUSH_KICK (NULL allowed otherwise). */
pic_status pic_push(pic_beam b, int kind, double value, const void* d_Ep, void* stream);

/* evolve(): n_steps split-operator steps, one per lattice slice (see pic_element), cycling over
 * the slices of lattice[0..n_el): the slice's first half map, the space-charge kick over the
 * slice length with the field of the positions at that point (geometry, deposit, IGF,
 * Poisson, field, gather), the second half map.  PIC_EINVAL for an unknown element kind, a
 * negative or non-finite length, a non-finite strength or nslice outside 1..1e6.  Updates X in place; the particle order
 * of X is preserved (internally the particles are binned by grid tile every step in two
 * workspace copies and returned to X in the caller's order at the end of the call).  With
 * desc.space_charge = 0 only the linear maps are applied.  If the device flags an error
 * during the call (see pic_check), X is left as it was before the call.  Bitwise reproducible:
 * the binned deposit sums each tile's charge window as 64-bit integers, exact in any order, and
 * forms the grid from the tiles in a fixed order; reductions have a fixed shape; so repeated
 * calls from the same state give the same bits although the order of particles within a tile
 * and of the atomics varies; the same holds for pic_track_batch, whose beams equal their
 * pic_track_n_steps results bit for bit.  (The slice-step diagnostics' moment sums are
 * reproducible to rounding only.)  Inside a call, a slice's second half map and the next
 * slice's first are applied as their product (the same linear map, rounded in another order);
 * the call's last step applies the second half map alone, so a run split into several calls
 * equals the same run in one call to rounding, not bit for bit. */
pic_status pic_track_n_steps(pic_beam b, const pic_element* lattice, int n_el, int n_steps,
                             void* stream);

/* evolve() without returning to the caller's particle order: as pic_track_n_steps, but X is left
 * in the order of the last step's binning (particles grouped by grid tile), which the next
 * call takes as its input.  d_ids (optional, device, n uint32, 4-byte aligned, caller-owned):
 * labels that travel with the particles: on return d_ids[i] is the label that was at the index
 * the particle now in slot i had on entry (start from 0..n-1 to follow the caller's indices;
 * NULL: no labels, 8 bytes less traffic per particle and step).  Per call this saves the
 * return to the caller's order at the end (the last step's gather-kick writes X directly) and,
 * when X is still in the order a previous binned call on this handle left it in, the move into
 * tile order on the first step, which then only ranks (the handle keeps that flag; the
 * pic_init_beam* calls clear it, and an X in any other order is only slower, never wrong); the
 * physics is the same, particle by particle and bit for bit, as pic_track_n_steps calls of
 * the same step counts (moments, the objective and the deposit do not depend on the order).  X is left as it was if the device
 * flags an error at any step's geometry (non-finite coordinate, zero-extent box). */
pic_status pic_track_n_steps_binned(pic_beam b, const pic_element* lattice, int n_el,
                                    int n_steps, uint32_t* d_ids, void* stream);

/* Slice-step diagnostics (Listing 1: set_slice_step_diagnostics(True)): as pic_track_n_steps,
 * and after every step j the moments of the particles at the end of that step go to the device
 * array d_diag[27*j .. 27*j+26] (27 * n_steps doubles, 8-byte aligned, caller-owned): the six
 * means of (x, px, y, py, z, delta), then the 21 centred second moments <d_a d_b> with 1/n, for
 * a <= b in row-major order of the upper triangle.  Each step then runs its gather-kick to
 * the end of the step and applies the next step's first half map in a separate pass (about
 * 190 B more HBM traffic per particle and step).  Results equal pic_track_n_steps' to rounding;
 * the moments of step j use the same reduction as pic_moments. */
pic_status pic_track_n_steps_diag(pic_beam b, const pic_element* lattice, int n_el, int n_steps,
                                  double* d_diag, void* stream);

/* Batched tracking of many independent beams (each created with pic_beam_create, all with the
 * same shape and grid precision, space_charge = 1; grids and particle counts may differ).
 * pic_batch_create copies the beams' device descriptors and their lattices (lattices[b] has
 * n_el[b] elements, expanded into slices and cycled over the steps as in pic_track_n_steps)
 * into the caller's workspace d_work
 * blocks_per_beam (1..65535, 0 = 256) is the workgroup count per beam of the binned deposit
 * and gather;
 * (pic_batch_workspace_bytes, 256-byte aligned) and synchronises `stream`.  The beams' handles,
 * arrays and workspaces must outlive the batch.
 * pic_track_batch runs n_steps steps of pic_track_n_steps on every beam, with one launch per
 * stage covering all beams; the whole n_steps loop is captured into one HIP graph on the first
 * call with that step count (on `stream`, which must not be the null stream) and replayed by
 * later calls.  Device errors are reported per beam by pic_check. */
size_t pic_batch_workspace_bytes(int n_beams, const pic_element* const* lattices,
                                 const int* n_el);
pic_status pic_batch_create(pic_beam* beams, int n_beams, const pic_element* const* lattices,
                            const int* n_el, int blocks_per_beam, void* d_work,
                            size_t work_bytes, void* stream, pic_batch* out);
pic_status pic_track_batch(pic_batch bt, int n_steps, void* stream);
pic_status pic_batch_destroy(pic_batch bt);

/* Workspace bytes of pic_track_adjoint for n_steps steps with a checkpoint every ckpt_every
 * steps (0 on invalid arguments). */
size_t pic_adjoint_workspace_bytes(const pic_beam_desc* d, int n_steps, int ckpt_every);

/* Reverse sweep (discrete adjoint) of n_steps steps of pic_track_n_steps.  The paper gives no
 * differentiation; its machine-learning coupling is only named (sections "Software Design",
 * "ImpactX").  Objective J = w[0] sigma_x + w[1] sigma_y + w[2] eps_x + w[3] eps_y of the final
 * beam (centred rms sizes and geometric emittances).  The gradient is that of the tracking as
 * pic_track_n_steps runs it, whose grid geometry follows the particles: every step's box
 * (min / max of the kick-point positions) sets origin and spacing, and the terms through them
 * (deposit and gather weights, the centred difference, the Green's function or field kernels'
 * dependence on the cell) reach the particles at the box's faces.  Where two particles tie for
 * a box face, the one with the lower index takes the term (the map has a kink there).
 * On entry X holds X0; on return X holds the final state (the forward pass, run in the
 * caller's particle order) and
 *   out_m[4]     (sigma_x, sigma_y, eps_x, eps_y) of the final state (host),
 *   dJ_dk[n_el]  dJ/dk of the lattice strengths, summed over the steps (slices) that use each:
 *                a thin element's k [1/m] enters its quad kick, a quadrupole's k [1/m^2] both
 *                half maps of each of its slices; drifts get 0 (host),
 *   d_lam        dJ/dX0, device array of 6*n doubles in the layout of X,
 *   dJ_dL[36]    if d_xi (device, 6*n draws with X0 = L xi) is given: dJ/dL = sum_i lam_i xi_i^T,
 *                row-major 6x6 (host); only the lower triangle is a parameter of L.
 * The forward states are checkpointed every ckpt_every steps in the caller's workspace
 * d_adj_work (pic_adjoint_workspace_bytes, 256-byte aligned) and recomputed per segment.
 * Lattices as for pic_track_n_steps (thin, drift and quadrupole elements, one step per slice).
 * With desc.direct_field the charge's adjoint goes through the transposed field convolutions.
 * Needs desc.space_charge = 1 and 1 <= n_el <= 1024.  Synchronises `stream`; returns the device error flag of any step
 * (PIC_EDOMAIN). */
pic_status pic_track_adjoint(pic_beam b, const pic_element* lattice, int n_el, int n_steps,
                             int ckpt_every, const double w[4], void* d_adj_work,
                             size_t adj_work_bytes, double* d_lam, const double* d_xi,
                             double out_m[4], double* dJ_dk, double dJ_dL[36], void* stream);

/* Beam statistics (paper: "beam statistics"): mean[6] and centred second moments cov[36]
 * (row-major, 1/n normalisation) of X.  Synchronises `stream`; PIC_EDOMAIN if the device
 * error flag is set. */
pic_status pic_moments(pic_beam b, double mean[6], double cov[36], void* stream);

/* The objective terms of pic_track_adjoint for the current X: out_m = (sigma_x, sigma_y, eps_x,
 * eps_y), the centred rms sizes and the geometric (unnormalised) emittances
 * eps_x = sqrt(<dx^2><dpx^2> - <dx dpx>^2), as the paper quotes emittance (sections "Usage
 * Example", "Benchmark: FODO Cell"), from the moments of pic_moments.  out_m is host memory.
 * Synchronises `stream`; PIC_EDOMAIN if the device error flag is set. */
pic_status pic_objective(pic_beam b, double out_m[4], void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid allocation): the beam statistics of pic_moments for a phase-space array
 * d_X (6*n doubles in the layout of X, device, 8-byte aligned, 1 <= n < 2^31) with no handle
 * and no workspace.  d_out (device, 27 doubles, 8-byte aligned, caller-owned) receives the six
 * means of (x, px, y, py, z, delta), then the 21 centred second moments <d_a d_b> (1/n) for
 * a <= b in row-major order of the upper triangle, the layout of pic_track_n_steps_diag; the
 * values equal pic_moments' bit for bit (same kernels, same reduction shape).  The reduction's
 * partial sums live in a fixed 221 KB device array inside the library (one per GPU, held
 * until the process ends); the call allocates nothing, does not synchronise and only enqueues
 * four kernels on `stream`.  Calls that overlap on one GPU (different streams without
 * ordering) race on that array.  PIC_EINVAL for a NULL or misaligned pointer or n outside
 * 1 .. 2^31 - 1; PIC_EHIP if a launch fails. */
pic_status pic_moments_noalloc(const double* d_X, int64_t n, double* d_out, void* stream);

/* Geometry of the last deposit: out[0..2] origin (x, y, z) [m], out[3..5] lab spacings,
 * out[6..8] rest-frame spacings (hx, hy, gamma hz).  Synchronises `stream`. */
pic_status pic_get_geometry(pic_beam b, double out[9], void* stream);

/* Stage timing of pic_track_n_steps (section "ImpactX" lists profiling among the shared PIC
 * routines).  pic_profile_start resets the counters and makes the following
 * pic_track_n_steps calls record a HIP event pair around every launch of each stage, on the
 * caller's stream; pic_profile_read synchronises those events, writes the summed milliseconds
 * and the number of launches per stage, and stops recording.  Stages:
 *   PIC_STAGE_PROLOGUE  thin quad + half drift of the first step, with the box reduction
 *   PIC_STAGE_GEOMETRY  grid geometry from the box, clearing of the charge grid
 *   PIC_STAGE_GREEN     integrated Green's function and its forward FFT
 *   PIC_STAGE_DEPOSIT   the charge-deposition kernel alone
 *   PIC_STAGE_SOLVE     zero padding, forward FFT, spectral product, inverse FFT, gradient
 *   PIC_STAGE_GKD       the fused gather, kick, drift (and next thin quad, half drift, box)
 *                       kernel alone
 *   PIC_STAGE_BIN       tile keys and histogram, scan and work list, counting-sort scatter
 *   PIC_STAGE_UNPERMUTE return of the particles to the caller's order and array */
enum {
  PIC_STAGE_PROLOGUE = 0, PIC_STAGE_GEOMETRY = 1, PIC_STAGE_GREEN = 2, PIC_STAGE_DEPOSIT = 3,
  PIC_STAGE_SOLVE = 4, PIC_STAGE_GKD = 5, PIC_STAGE_BIN = 6, PIC_STAGE_UNPERMUTE = 7,
  PIC_NSTAGES = 8
};
pic_status pic_profile_start(pic_beam b);
pic_status pic_profile_read(pic_beam b, double ms[8], int64_t launches[8]);

/* Synchronise `stream` and report the device error flag (PIC_OK or PIC_EDOMAIN). */
pic_status pic_check(pic_beam b, void* stream);

/* Message for the last failure on the calling thread ("" if none). */
const char* pic_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PIC_H */
