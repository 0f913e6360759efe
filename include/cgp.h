/*
 * cgp.h -- C ABI of the MI355X (gfx950) coarse-grid-projection (CGP) QG time step.
 *
 * Method: O. San and A. E. Staples, "An Efficient Coarse Grid Projection
 * Method for Quasigeostrophic Models of Large-Scale Ocean Circulation"
 * (arXiv 1308.3290).  One CGPRK3 step (Sec. 3.2) advances the relative
 * vorticity of the one-layer barotropic model (Sec. 2.1) or the two-layer
 * stratified model (Sec. 2.2) on a rectangular beta-plane basin with free-slip
 * walls.  Each of the three TVD-RK3 stages (Sec. 4.2):
 *   (ii)  restricts the fine vorticity to the coarse grid by full weighting,
 *         level times (Sec. 3.1);
 *   (iii) solves the coarse elliptic problem with sine transforms and a
 *         diagonal eigenvalue divide (Sec. 4.3); for two layers the coupled
 *         problem is split into a barotropic Poisson and a baroclinic
 *         Helmholtz problem (equivalent to that section's 2x2 per-mode solve);
 *   (iv)  prolongs psi bilinearly back to the fine grid (Sec. 3.1);
 *   (i)   updates the vorticity on the fine grid with the Arakawa Jacobian
 *         (Sec. 4.1), the beta term, Laplacian eddy viscosity and the forcing.
 *
 * Conventions shared by every call
 *   - nx, ny count grid INTERVALS: nodes i = 0..nx, j = 0..ny (Sec. 4.4 index
 *     ranges).  Node arrays are y-major with x contiguous, element (j, i) at
 *     j*(nx+1) + i; two-layer arrays are [2][ny+1][nx+1], layer 1 (top) first.
 *   - Prognostic variable: omega = Laplacian(psi) (one layer, Sec. 2.1) or
 *     Q_i = Laplacian(psi_i) + F_i (psi_j - psi_i) (two layers, Sec. 2.2):
 *     the potential vorticity with the planetary part y removed and divided
 *     by Ro.  The step solves Laplacian_h psi = omega on the coarse grid.
 *   - Walls: psi = 0 and omega = 0 on the boundary ring (Sec. 2.1, 2.2).
 *     Input rings are treated as zero whatever they hold; every output ring
 *     is written as zero.  The forcing ring is ignored.
 *   - Memory: every pointer argument named *_dev is DEVICE memory owned by the
 *     caller; the library never allocates device memory.  The workspace given
 *     to a create call belongs to the handle until cgp_destroy and must not be
 *     touched meanwhile.  Host pointers are read during the call only.
 *   - Streams: `stream` is a hipStream_t passed as void* (NULL = the null
 *     stream).  All device work is enqueued asynchronously on it; no call
 *     synchronises the host except where stated.  A handle is not thread
 *     safe; two calls on one handle must not overlap in time on the device.
 *   - Errors: every call returns a cgp_status; nothing aborts or throws
 *     across the ABI.  cgp_last_error() gives a message for the calling
 *     thread's most recent failure.  Invalid sizes, pointers or parameters give
 *     CGP_ERR_INVALID, sizes outside the supported set CGP_ERR_UNSUPPORTED,
 *     HIP failures CGP_ERR_DEVICE.
 */
#ifndef CGP_H
#define CGP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CGP_OK = 0,
  CGP_ERR_INVALID = 1,
  CGP_ERR_UNSUPPORTED = 2,
  CGP_ERR_DEVICE = 3,
  CGP_ERR_NONFINITE = 4
} cgp_status;

typedef enum { CGP_F32 = 0, CGP_F64 = 1 } cgp_dtype;

/* One basin.  Vorticity-form coefficients: dividing the nondimensional
 * equations of Sec. 2.1 / 2.2 by Ro gives
 *   one layer:  d omega/dt = -J(psi, omega) - inv_ro J(psi, y) + inv_re Lap(omega) + F
 *   two layers: d Q_i/dt  = -J(psi_i, Q_i) - inv_ro J(psi_i, y) + inv_re Lap(zeta_i)
 *                           + [i=1] F - [i=2] drag zeta_2,
 *               zeta_i = Q_i - F_i (psi_j - psi_i),
 * with inv_ro = 1/Ro, inv_re = 1/Re (= A/Ro for two layers), f1 = Fr/(Ro delta),
 * f2 = Fr/(Ro (1 - delta)), drag = sigma/Ro.  Supported sizes: level >= 0,
 * nx and ny divisible by 2^level, and the coarse interval counts
 * Mx = nx/2^level, My = ny/2^level each of the form 2^k or 3*2^k with
 * 4 <= M <= 1024; two layers with coarsening need Mx <= 512. */
typedef struct cgp_config {
  int32_t nx, ny;      /* fine grid intervals */
  int32_t level;       /* coarsening level l; factor 2^l; 0 = plain full-grid step */
  int32_t nlayers;     /* 1 or 2 */
  int32_t dtype;       /* cgp_dtype: arithmetic and storage type of every field */
  int32_t reserved;    /* must be 0 */
  double lx, ly, y0;   /* basin [0, lx] x [y0, y0 + ly] */
  double inv_re, inv_ro;
  double f1, f2, drag; /* two-layer coefficients, ignored for one layer */
  double dt;           /* time step; with cfl > 0 the largest (and first) step */
  double cfl;          /* CFL number c of Sec. 4.2: 0 keeps dt fixed; c > 0 adapts
                        * the step: after every step, the next step's size is
                        * min(dt, c min(dx, dy) / max |grad psi|), the maximum of
                        * |d psi/dx| and |d psi/dy| (centred differences at the
                        * interior nodes, every layer) taken on the prolonged psi
                        * of the step's third stage (dt itself when that maximum
                        * is 0).  The step state lives in the workspace, so that
                        * a run split over calls takes the same steps. */
  int32_t solver;      /* coarse elliptic solver: 0 = sine transform (Sec. 4.3, exact);
                        * 1 = multigrid V(2,2) cycles (red-black Gauss-Seidel,
                        * full weighting, bilinear interpolation, exact coarsest
                        * grid), an iterative black box under CGP: one layer,
                        * single basin, no adjoint */
  int32_t mg_cycles;   /* V-cycles per solve with solver 1 (0: 12; each cycle cuts
                        * the residual about tenfold) */
  int32_t fused_rows;  /* one layer at coarsening factor 2: coarse rows per block of the
                        * fused stage pass, 0 (the default, 2) or 4.  A block
                        * synthesises its rows and one on each side, and recomputes
                        * one fine row below its own: 4 rows per block transform 6
                        * coarse rows for 4 owned instead of 4 for 2 and recompute 1
                        * fine row in 9 instead of 1 in 5, in half the blocks.
                        * Faster for large FP32 ensembles (two blocks still fit a
                        * CU), slower for single basins (half the CUs) and FP64
                        * ensembles (one block per CU); both give the same bits.
                        * Shared by every member of a handle; ignored elsewhere.  The
                        * persistent launch (cgp_set_launch mode 1) needs 2. */
} cgp_config;

typedef struct cgp_handle cgp_handle;

/* How a handle's time steps are launched (cgp_set_launch).  mode 0: every
 * pass of a stage is its own launch (one per group of members of one
 * transform length; captured steps run the groups' chains on forked
 * streams).  mode 1: ONE persistent launch per RK3 stage over every member:
 * workgroups take tiles of work from a queue in the workspace (first every
 * member's pass-B column pairs, b_tile per tile, then its fused-pass row
 * blocks, f_tile per tile), and per-member counters make a member's fused
 * tiles wait until its pass B is done.  Mode 1 needs one layer and every
 * member at coarsening factor 2 with row transforms of 128, 256, 384 or 512
 * points and column transforms of 256, 512, 768 or 1024 points (rows of at
 * most 256 intervals, 128 x 256 up to 512 x 1024 grids).  wg_per_cu: the
 * launch grid's workgroups per compute unit (0: as many as can be
 * resident).  Both modes give the same bits. */
typedef struct cgp_launch {
  int32_t mode;
  int32_t b_tile;
  int32_t f_tile;
  int32_t wg_per_cu;
} cgp_launch;

/* Bytes of device workspace a single-basin handle needs.  Host only. */
cgp_status cgp_workspace_size(const cgp_config* cfg, size_t* bytes);

/* Create a single-basin handle.  Builds the FP64 sine/cosine and eigenvalue
 * tables (Sec. 4.3) on the host and uploads them into workspace_dev on
 * `stream`.  workspace_dev must be 256-byte aligned and at least
 * cgp_workspace_size bytes. */
cgp_status cgp_create(const cgp_config* cfg, void* workspace_dev, size_t bytes,
                      void* stream, cgp_handle** out);

/* Release the handle's host state.  The workspace goes back to the caller
 * once work enqueued on the handle has finished.  The handle's captured
 * graphs are destroyed after the last replay it enqueued has finished (the
 * call waits for that replay, not for other work). */
cgp_status cgp_destroy(cgp_handle* h);

/* Advance omega_dev ([L][ny+1][nx+1], in/out) by nsteps CGPRK3 steps
 * (Sec. 3.2 listing: three restrict-solve-prolong cycles and three fine-grid
 * updates per step).  forcing_dev is the wind-forcing field F
 * ([ny+1][nx+1], vorticity units, layer 1 only), e.g. inv_ro*sin(pi*y).
 * psi_out_dev (nullable, [L][ny+1][nx+1]): if set, receives
 * psi = P^l L_c^-1 R^l omega of the final state.  nsteps >= 0. */
cgp_status cgp_step(cgp_handle* h, void* omega_dev, const void* forcing_dev,
                    void* psi_out_dev, int32_t nsteps, void* stream);

/* cgp_step for callers that cannot allocate device memory (tight serving
 * loops, harnesses that forbid hipMalloc or any device allocation): the
 * same kernels on the same arrays as cgp_create + cgp_step + cgp_destroy of a
 * fresh single-basin handle, with the workspace in a static device array of
 * the library (48 MiB on each GPU it runs on, held until the process ends)
 * instead of a caller workspace.  The caller passes cfg (host), omega_dev
 * (in/out), forcing_dev and psi_out_dev (nullable) exactly as for cgp_step.
 * No call allocates device memory: the library takes the array's address
 * with hipGetSymbolAddress at its first call on a device.  Every call
 * uploads the handle tables and a fresh step state into the array (the model
 * time of cgp_time_state restarts at 0; with cfl > 0 the first step is dt)
 * and synchronises `stream` once after that upload, so it cannot itself be
 * captured into a graph.  Configurations whose workspace (cgp_workspace_size)
 * exceeds 48 MiB give CGP_ERR_INVALID before any device work; every
 * 512 x 1024 one- and two-layer FP64 configuration fits.  All calls on one
 * GPU share the array: calls that overlap in time on one GPU (two streams,
 * two host threads) race and must be serialised by the caller. */
cgp_status cgp_step_noalloc(const cgp_config* cfg, void* omega_dev, const void* forcing_dev,
                            void* psi_out_dev, int32_t nsteps, void* stream);

/* Step state: out_dev[2m] = the dt of member m's latest step (the configured
 * dt before the first step), out_dev[2m+1] = the model time its steps have
 * advanced since cgp_create (m = 0 for a single basin).  out_dev holds
 * 2 * members doubles (device memory), written on `stream`. */
cgp_status cgp_time_state(cgp_handle* h, double* out_dev, void* stream);

/* cgp_step (without psi_out) that also adds, after every step, dt * omega of
 * the new state to sum_dev (FP64, the handle's field layout; dt of that step):
 * the time integral of omega over the steps, from which the time mean of
 * omega, and by linearity of the elliptic map that of psi, follow (the
 * statistics of the paper's long runs, Sec. 5.1).  Works for ensembles too
 * (packed fields).  use_graph != 0 replays captured graphs of the steps and
 * their sums (on a non-default stream). */
cgp_status cgp_step_mean(cgp_handle* h, void* omega_dev, const void* forcing_dev, int32_t nsteps,
                         double* sum_dev, int32_t use_graph, void* stream);

/* Running sums for time means (the statistics of the paper's long runs,
 * Sec. 5.1): sum_dev[k] += weight * w_m * field_dev[k] for every element k
 * of the handle's field layout (all members and layers, packed as
 * cgp_step's fields), in FP64 whatever the handle's dtype; w_m is the dt of
 * member m's latest step when times_dt != 0 (a time-weighted sum), else 1.
 * sum_dev holds that many doubles (device memory). */
cgp_status cgp_accumulate(cgp_handle* h, const void* field_dev, double* sum_dev, double weight,
                          int32_t times_dt, void* stream);

/* The CGP elliptic map alone: psi_dev = P^l L_c^-1 R^l omega_dev
 * (Sec. 3 steps (ii)-(iv); for two layers the coupled solve of Sec. 4.3).
 * Arrays [L][ny+1][nx+1]. */
cgp_status cgp_solve(cgp_handle* h, const void* omega_dev, void* psi_dev, void* stream);

/* Domain-averaged diagnostics of a state: out_dev[2*l] = E_l =
 * 1/(2A) sum over grid links of |forward difference of psi_l|^2 dx dy
 * (eq. 26 divided by the basin area A), out_dev[2*l+1] = Z_l = 1/(2A) sum of
 * omega_l^2 dx dy over interior nodes.  out_dev holds 2*L doubles (FP64
 * accumulation in a fixed order, so the result is deterministic). */
cgp_status cgp_diagnostics(cgp_handle* h, const void* omega_dev, const void* psi_dev,
                           double* out_dev, void* stream);

/* flag_dev (one int32 on the device) is set to 1 if any of the count
 * elements of field_dev (the handle's dtype) is NaN or infinite, else 0. */
cgp_status cgp_check_finite(cgp_handle* h, const void* field_dev, int64_t count,
                            int32_t* flag_dev, void* stream);

/* The same check, synchronous: CGP_OK if the count elements of field_dev
 * (the handle's dtype) are all finite, CGP_ERR_NONFINITE if any is NaN or
 * infinite.  Synchronises `stream`; the flag lives in the handle's
 * workspace, so this call is not graph-capturable and must not overlap other
 * work on the handle.  The time step itself never reads back. */
cgp_status cgp_assert_finite(cgp_handle* h, const void* field_dev, int64_t count, void* stream);

/* ------------------------------------------------------------------------
 * Adjoint (one-layer, FP64).  For w_{s+1} = a_s w_n + b_s (w_s + dt G(w_s)),
 * (a, b) = (0, 1), (3/4, 1/4), (1/3, 2/3), the adjoint reverses the stages:
 *   mu = b_s dt lam_{s+1};  g_F += mu;  acc_n += a_s lam_{s+1};
 *   lam_s = b_s lam_{s+1} + J(psi_s, mu) + inv_re Lap(mu)
 *           + A_l[ -J(omega_s, mu) + inv_ro J(mu, y) ],
 * using (J(psi,.))^T = -J(psi,.), (J(., omega))^T = J(omega, .), the skew
 * beta stencil and the symmetry of A_l = P^l L_c^-1 R^l (P = 4 R^T per level
 * in plain sums).  The tape holds the recomputed stage states.
 * ---------------------------------------------------------------------- */

/* Bytes of device tape cgp_adjoint_step needs for a segment of nsteps.
 * The adjoint differentiates steps of fixed size: cfl must be 0
 * (CGP_ERR_UNSUPPORTED otherwise, here and in cgp_adjoint_step). */
cgp_status cgp_tape_size(const cgp_config* cfg, int32_t nsteps, size_t* bytes);

/* Reverse sweep over one segment of nsteps >= 1 steps that starts from the
 * state omega_n_dev.  The forward states of the segment are recomputed into
 * tape_dev; then, on entry lambda_dev holds dL/d omega_{n+nsteps} and on exit
 * dL/d omega_n, and grad_forcing_dev ([ny+1][nx+1]) is INCREMENTED by the
 * segment's dL/dF.  All FP64, one layer only. */
cgp_status cgp_adjoint_step(cgp_handle* h, const void* omega_n_dev, const void* forcing_dev,
                            int32_t nsteps, void* lambda_dev, void* grad_forcing_dev,
                            void* tape_dev, size_t tape_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Ensembles: independent basins of uneven size and coefficients advanced
 * together, each pass of a stage one launch over every member.  A single
 * basin is an ensemble of one.  All members share the dtype and nlayers.
 * Packed arrays hold member m's [L][ny_m+1][nx_m+1] field at element offset
 * offsets[m] (cgp_ensemble_offsets), members in order, no gaps.
 * ---------------------------------------------------------------------- */
cgp_status cgp_ensemble_offsets(const cgp_config* members, int32_t count, int64_t* offsets_host,
                                int64_t* total_elements);
cgp_status cgp_ensemble_workspace_size(const cgp_config* members, int32_t count, size_t* bytes);
cgp_status cgp_ensemble_create(const cgp_config* members, int32_t count, void* workspace_dev,
                               size_t bytes, void* stream, cgp_handle** out);
/* Advance every member by nsteps.  With use_graph != 0 the step is captured
 * once into a HIP graph (per pointer set) and replayed nsteps times; only
 * graphs run the transform-length chains of an ensemble concurrently.  For a
 * single basin direct launches (use_graph = 0) measured faster on MI355X:
 * graph kernel nodes there do not get the kernel arguments preloaded. */
cgp_status cgp_ensemble_step(cgp_handle* h, void* omega_packed_dev,
                             const void* forcing_packed_dev, int32_t nsteps, int32_t use_graph,
                             void* stream);

/* Select how h's time steps are launched (cgp_launch; the default is mode 0
 * with tiles of 1).  Mode 1 on a handle without it gives
 * CGP_ERR_UNSUPPORTED; tiles below 1 or wg_per_cu outside 0..16,
 * CGP_ERR_INVALID.  Graphs captured before are dropped once the last replay
 * the handle enqueued has finished (the call waits for it); then the work
 * queue of mode 1 is uploaded into the workspace on `stream`, which is
 * synchronised. */
cgp_status cgp_set_launch(cgp_handle* h, const cgp_launch* launch, void* stream);

/* The handle's launch setting; *persistent_available (nullable) = 1 when
 * the handle can take mode 1.  Host only. */
cgp_status cgp_get_launch(cgp_handle* h, cgp_launch* launch, int32_t* persistent_available);

/* The sticky fault flag of mode 1 (host memory): 1 if a fused tile ever
 * stopped waiting for its member's pass B after its bounded number of polls
 * (its results are then wrong), else 0.  Synchronises `stream`. */
cgp_status cgp_persistent_fault(cgp_handle* h, int32_t* flag_host, void* stream);

/* Measurement.  Times each pass of one RK3 stage on the handle's current
 * workspace contents: pass 0 (restriction + x transform of omega_dev),
 * 1 (y transforms + eigenvalue divide), 2 (x transform + prolongation into
 * psi), 3 (Arakawa right-hand side + RK3 combine in the form of stage 2:
 * reads stage 1, psi, the forcing and omega_dev, writes stage 2), 4 (the
 * fused form of passes 2 and 3 that one-layer time steps use when every
 * member's rows hold at most 512 intervals and 2^level <= 8) and 5 (pass 4
 * followed by pass 0 of the next stage on its result, the form time steps
 * launch); 0 is reported for 4 and 5 on handles without them.  Each pass is
 * launched `reps` times back to back on `stream` between two HIP events;
 * ms_host[p] (6 doubles, host memory) receives the mean milliseconds per
 * launch.  Synchronises the stream.  omega_dev is only read. */
cgp_status cgp_time_passes(cgp_handle* h, const void* omega_dev, const void* forcing_dev,
                           int32_t reps, double* ms_host, void* stream);

/* Measurement in the context of a time step.  Advances omega_dev by nsteps
 * (1..4096) steps with direct launches, exactly as cgp_step does (pass A of
 * the initial state, then per stage pass B and the fused stage pass with the
 * next stage's restriction and x transform), with a HIP event recorded on
 * `stream` before and after each of those launches.  ms_host (3 doubles,
 * host memory) receives the mean milliseconds per launch of pass B, the mean
 * per launch of the fused pass, and the mean milliseconds per step of the
 * whole run (events included).  Synchronises the stream.  Handles whose
 * steps do not use the fused pass give CGP_ERR_UNSUPPORTED. */
cgp_status cgp_time_step_passes(cgp_handle* h, void* omega_dev, const void* forcing_dev,
                                int32_t nsteps, double* ms_host, void* stream);

/* Measurement build only: exported by libcgp_stamps.so, the library built
 * with CGP_PHASE_STAMPS (libcgp.so does not have it).  In that build thread 0
 * of every block of a pass-B launch and of a one-layer fused stage pass
 * launch writes the device's steady clock at its phase boundaries (the
 * arithmetic is unchanged; the persistent stage kernel of ensembles writes
 * no stamps); each launch overwrites the stamps of its blocks.  Copies the
 * stamps of the last launch of pass B (kind 0) or of the fused pass (kind
 * 1) to host_out: nblocks (1..4096, hardware block index order) x 8 slots of
 * uint64 clock ticks, unwritten slots unspecified.  Pass B slots: 0 block
 * start, 1 columns loaded, 2 forward transform and divide done, 3 results
 * stored.  Fused pass slots: 0 block start, 1 spectra in LDS, 2 inverse x
 * transform done, 3 vorticity tile in LDS, 4 stencil and RK3 combine done,
 * 5 restriction done, 6 block end.  *clock_khz (if not NULL) receives the
 * clock's rate.  Synchronises the device.  Bad kind, pointer or count:
 * CGP_ERR_INVALID. */
cgp_status cgp_phase_stamps(int32_t kind, uint64_t* host_out, int32_t nblocks,
                            int32_t* clock_khz);

/* Message for the calling thread's last failure ("" if none). */
const char* cgp_last_error(void);

/* Library version string. */
const char* cgp_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CGP_H */
