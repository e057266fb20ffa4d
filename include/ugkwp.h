/*
 * ugkwp.h - C ABI of the MI355X (gfx950) library for the hot path of one
 * UGKWP-LTS time step (Guo, Cao, Long, Xu, arXiv 2607.09552, Secs. III-IV).
 *
 * One call to ugkwp_step advances every cell by its own fixed local time step
 * (Eq. (33)), doing on the GPU:
 *   - the wave-particle decomposition W = W^h + W^p (Eq. (24)) with the LTS
 *     collisionless fraction e^{-dt_i/tau_i} and resampling of new particles
 *     (Eqs. (25)-(26), Sec. IV.B);
 *   - the free-transport time of retained particles (Eq. (51));
 *   - free transport and tracking through the mesh with mass and remaining
 *     time scaled by dt_R/dt_L at every crossing (Eqs. (41), (52));
 *   - the before/after particle tally (Eqs. (29)-(30)) and removal of
 *     collided particles, with the store re-sorted by cell;
 *   - the time-averaged equilibrium and analytic free-transport wave fluxes
 *     (Eqs. (49)-(50)) on every face;
 *   - the conservative update (Eq. (53)).
 *
 * Conventions for every call:
 *   - Units are nondimensional; layouts are row-major [item][component];
 *     W = (rho, rho U_x[, rho U_y], rho E) has dim + 2 components.
 *   - Ownership: every input array is copied at init; the caller keeps it.
 *     Outputs go to caller buffers (host unless the name says device).
 *   - All GPU work is ordered on the stream given at init (NULL = the
 *     library's own stream).  Within a step, the face fluxes run on a side
 *     stream that the context creates (default priority); it waits on an
 *     event of the given stream and the given stream waits on it before
 *     the update, so work enqueued later on the given stream, its
 *     synchronization and graph capture of it include the side work.
 *     Getters synchronize the given stream.
 *   - A context is not thread-safe; separate contexts are independent.
 *   - Every call returns UGKWP_OK or a negative error code;
 *     ugkwp_last_error() gives a text.  A step that fails (ENUMERIC,
 *     EOVERFLOW) is not committed: the fields, the particle set, its tallies,
 *     the running averages and the step counter stay those of the last
 *     committed step, and the context can be used on (for instance saved,
 *     or stepped again after a change of tuning).  One exception: a
 *     residual term outside its summation window (a one-step density change
 *     some 2^12 times the initial maximum density) is found after the
 *     fields were updated; that step stays committed and the call returns
 *     ENUMERIC after it.
 *   - The particle tallies (Eqs. (24), (29)-(30)), the wall impulses and the
 *     residual sums are exact fixed-point sums (every term cut into 32-bit
 *     chunks of a window fixed at init: six for tallies and wall impulses,
 *     four for the residual sums) rounded once to FP64, so every result is
 *     reproducible bit for bit from run to run, whatever order the GPU's
 *     atomics take.
 *   - The library requires a gfx950 device; it has no CPU fallback.
 */
#ifndef UGKWP_H
#define UGKWP_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

enum {
  UGKWP_OK = 0,
  UGKWP_EINVAL = -1,    /* bad argument, mesh or parameter */
  UGKWP_ENOMEM = -2,    /* device or host allocation failed */
  UGKWP_EDEVICE = -3,   /* HIP runtime error or no usable device */
  UGKWP_EOVERFLOW = -4, /* particle capacity or a caller buffer too small */
  UGKWP_ENUMERIC = -5,  /* non-finite or invalid state, runaway tracking */
  UGKWP_ESTATE = -6,    /* call not valid in the current state */
  UGKWP_EIO = -7        /* a checkpoint file could not be written or read */
};

enum { /* boundary face types */
  UGKWP_BC_FARFIELD = 1,     /* fixed ghost state; injects particles */
  UGKWP_BC_OUTFLOW = 2,      /* ghost = copy of the interior cell; injects */
  UGKWP_BC_WALL_DIFFUSE = 3, /* isothermal wall, diffuse reflection */
  UGKWP_BC_SYMMETRY = 4,     /* mirror ghost, specular particles */
  UGKWP_BC_WALL_MAXWELL = 6  /* isothermal wall with accommodation alpha (Sec. V.B):
                                a hit re-emits diffusely with probability alpha,
                                else reflects specularly; wave flux alpha times
                                the diffuse wall's plus (1 - alpha) times the
                                mirror flux */
};

typedef struct ugkwp_ctx ugkwp_ctx;

/* Mesh of cells Omega_i with faces s_j and unit normals n_j (Sec. III). */
typedef struct {
  int32_t dim;                /* 1 or 2 */
  int64_t n_nodes;
  const double *nodes;        /* [n_nodes*dim]; 1D: increasing x_0..x_N */
  int64_t n_cells;            /* 1D: n_nodes - 1 */
  const int64_t *cell_ptr;    /* 2D: CSR of strictly convex CCW polygons (3..8 vertices); NULL in 1D */
  const int64_t *cell_nodes;  /* 2D: node ids, [cell_ptr[n_cells]] */
  int64_t n_bfaces;           /* every open edge (2D) / both end nodes (1D) */
  const int64_t *bface_nodes; /* [n_bfaces*dim] node ids of each boundary face */
  const int32_t *bface_type;  /* UGKWP_BC_* */
  const double *bface_data;   /* [n_bfaces*8]: far field rho, U_x, U_y, T; wall T_w;
                                 Maxwell wall T_w, alpha; else unused */
} ugkwp_mesh;

/* Gas (Sec. II: tau = mu/p, mu = mu_ref (T/T_ref)^omega), time stepping
 * (Eq. (33) CFL number, Eq. (34) GTS when lts = 0), sampling (Eq. (26) N_ref),
 * the Philox seed, and the freestream used for C_p, C_F, C_Q, C_d (Sec. V). */
typedef struct {
  double R, omega, mu_ref, T_ref, Pr;
  int32_t D;                  /* internal degrees of freedom (0: monatomic, up to 64); particles then carry |xi|^2 / 2 */
  double cfl;
  int32_t n_ref;
  int32_t lts;                /* 1 local time steps, 0 global dt_G = min dt_i */
  uint64_t seed;
  double rho_inf, u_inf_x, u_inf_y, T_inf, L_ref;
  int64_t particle_capacity;  /* 0 = automatic; grows on demand */
  void *stream;               /* hipStream_t or NULL */
  int32_t precision;          /* 0: FP64 particles (the parity path); 1: mixed,
                                 particle positions (relative to the cell's
                                 centroid) and velocities in FP32, masses,
                                 tallies, cells and fluxes in FP64 */
  int32_t wave_only;          /* 1: E = 0 -- no particles, the free-transport wave
                                 carries all of g^h (the gas-kinetic scheme of the
                                 coarse solves behind a warm start); 0: UGKWP */
  int32_t dt_source;          /* state Eq. (33) takes dt_i from: 0 the initial
                                 field W0 (Sec. IV.B), 1 the freestream reference
                                 (rho_inf, u_inf, T_inf) in every cell, so that
                                 runs from different initial fields share one
                                 set of time steps */
} ugkwp_params;

/* Builds faces and geometry, uploads the state and computes the local time
 * steps dt_i from W0 (Eq. (33); from the freestream when dt_source = 1),
 * fixed for the whole run; the particle set
 * starts empty (W^p = 0, Sec. III.C).  W0 is [n_cells*(dim+2)] host memory.
 * Sizes: fewer than 2^28 cells in a context (2^24 cells plus boundary
 * faces per case, the particle ids' layout).
 * Errors: EINVAL (mesh not matching its boundary list, non-convex or
 * clockwise cell, bad parameters, sizes), ENUMERIC (invalid W0), EDEVICE,
 * ENOMEM.  On an error *out still holds a context (NULL only when out is
 * NULL or the context itself could not be allocated): ugkwp_last_error()
 * on it says why, and the caller frees it with ugkwp_free; no other call
 * may use it.  Arguments are checked before any device call. */
int ugkwp_init(const ugkwp_mesh *mesh, const ugkwp_params *params, const double *W0, ugkwp_ctx **out);

/* A batch of independent cases in one context: the cases' meshes are joined
 * into one disjoint mesh and every step advances all of them together.  Each
 * case is computed exactly as if alone with its own parameters: its particle
 * ids use its own cell and boundary-face numbering and its random numbers its
 * own seed, so case k of a batch gives the results of ugkwp_init with
 * meshes[k], params[k], W0[k].  All cases must share dim (2), the gas (R,
 * omega, T_ref, Pr, D), cfl, n_ref, lts, precision and stream; mu_ref, seed,
 * the freestream reference, dt_source and capacity may differ.  W0[k] is
 * [meshes[k].n_cells*4].  Errors as ugkwp_init, EINVAL for mismatched shared
 * parameters. */
int ugkwp_init_batch(int32_t n_cases, const ugkwp_mesh *meshes, const ugkwp_params *params,
                     const double *const *W0, ugkwp_ctx **out);
/* Cell range of case k in the joined mesh (fields and particles of the batch
 * are indexed by it) and its range in the list of wall faces. */
int ugkwp_case_range(ugkwp_ctx *ctx, int32_t case_id, int64_t *first_cell, int64_t *n_cells, int64_t *first_wall,
                     int64_t *n_wall);
/* Residuals (as ugkwp_residual) and wall quantities (as ugkwp_surface) of one
 * case of a batch. */
int ugkwp_case_residual(ugkwp_ctx *ctx, int32_t case_id, double *r_inst, double *r_avg);
int ugkwp_case_surface(ugkwp_ctx *ctx, int32_t case_id, int32_t mode, double *out, int64_t cap, int64_t *n_wall,
                       double *Cd);

/* Advances n_steps UGKWP-LTS steps (Secs. III.C, IV.B).  Errors: ENUMERIC
 * (invalid cell state at the start of a step, runaway tracking), EOVERFLOW
 * (more than 2^20 particles born in one cell), ENOMEM, EDEVICE. */
int ugkwp_step(ugkwp_ctx *ctx, int32_t n_steps);

/* ugkwp_step for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation):
 * the same steps with the same results, bit for bit, but the step's
 * accumulators (the per-cell histogram and scatter cursors of the re-sort,
 * the wall-impulse and residual chunks, counters and the scan's block sums)
 * live in one static device array of 48 MiB that the library holds on each
 * device it runs on until the process ends, and the call allocates nothing:
 * no store growth (EOVERFLOW if the step would need more particle slots
 * than the store holds: give ugkwp_params.particle_capacity, or let
 * ugkwp_step grow it first), no graph capture (every kernel launched
 * directly), no timing events (ESTATE while ugkwp_profile is on).
 * EOVERFLOW if the mesh's accumulators exceed the array (about 24 bytes per
 * cell: meshes up to some 1.9 million cells).  Every call on a device
 * shares that device's array, which keeps the last call's contents (each
 * step clears what must start at zero): calls that overlap on one device,
 * from any context or thread, race.  Other errors as ugkwp_step. */
int ugkwp_step_noalloc(ugkwp_ctx *ctx, int32_t n_steps);

/* Advances until the residual target is met: stops after the first step
 * n >= 100 whose r_avg (see ugkwp_residual; every case's for a batch) is
 * below target (the convergence rule used for time-to-residual), or after
 * max_steps steps.  Wave-only runs (params.wave_only) test r_inst instead:
 * they carry no particle noise.  *converged = 1 if the target was met; the
 * step count is that of ugkwp_residual.  The test runs on the device after
 * every step.  Errors as ugkwp_step; EINVAL if target <= 0. */
int ugkwp_step_until(ugkwp_ctx *ctx, double target, int32_t max_steps, int32_t *converged);

/* Residuals after the last step (the paper defines none; reading): r_inst is
 * the area-weighted RMS of the last density change over rho_inf, r_avg the
 * same for the running mean of the density over all steps.  step = steps done.
 * For a batch: the largest over the cases. */
int ugkwp_residual(ugkwp_ctx *ctx, double *r_inst, double *r_avg, int64_t *step);

/* Wall quantities of Sec. V (diffuse and Maxwell wall faces in boundary-list order):
 * out[w*6 + 0..5] = face midpoint x, y, length, C_p, C_F, C_Q, and the drag
 * coefficient C_d = F_d / (rho_inf U_inf^2 L_ref / 2) (Sec. V.B).
 * mode 0: last step; 1: mean over all steps; 2: exponential moving average
 * with alpha = 2/1001 (Sec. V.A).  out may be NULL to query n_wall.
 * For a batch: case 0 (see ugkwp_case_surface).
 * Errors: ESTATE before the first step, EOVERFLOW if cap < n_wall. */
int ugkwp_surface(ugkwp_ctx *ctx, int32_t mode, double *out, int64_t cap, int64_t *n_wall, double *Cd);

/* Host copy of W, [n_cells*(dim+2)]. */
int ugkwp_get_fields(ugkwp_ctx *ctx, double *W);
/* Stream-ordered device-to-device copy of W into d_W (device pointer). */
int ugkwp_get_fields_device(ugkwp_ctx *ctx, void *d_W);
/* Local time steps dt_i, [n_cells]. */
int ugkwp_get_dt(ugkwp_ctx *ctx, double *dt);
/* Retained particles per cell after the last committed step and that
 * step's totals: transported (retained + new + entered from ghosts), new,
 * removed (collided), exited, and cells reset by the vacuum guard.  Any
 * pointer may be NULL. */
int ugkwp_get_counts(ugkwp_ctx *ctx, int32_t *count, int64_t *n_total, int64_t *n_new, int64_t *n_removed,
                     int64_t *n_exited, int64_t *n_guard);
/* Running sum over every committed step of the particles transported in it
 * (the n_total of ugkwp_get_counts, summed): the work counter behind the
 * particle-update rate.  Starts at 0 at init. */
int ugkwp_get_work(ugkwp_ctx *ctx, int64_t *n_transported);
/* Retained particles sorted by pid (then by cell: each case of a batch
 * numbers its particles on its own): pid = step << 44 | birth cell << 20 | j
 * (birth cell >= n_cells marks a boundary face), cell, mass, position
 * [n*dim], velocity [n*3], internal energy per unit mass |xi|^2 / 2 [n]
 * (0 when D = 0).  Pointers may be NULL; *n is set even when cap is too
 * small (then EOVERFLOW). */
int ugkwp_get_particles(ugkwp_ctx *ctx, int64_t cap, uint64_t *pid, int32_t *cell, double *m, double *x,
                        double *u, double *ei, int64_t *n);
/* Replaces the retained set (host arrays as in ugkwp_get_particles; ei may
 * be NULL: zero internal energy). */
int ugkwp_set_particles(ugkwp_ctx *ctx, int64_t n, const uint64_t *pid, const int32_t *cell, const double *m,
                        const double *x, const double *u, const double *ei);
/* Replace W ([n_cells*(dim+2)] host; the local time steps stay those of
 * the initial field, Eq. (33)); the density of the last step (behind
 * r_inst) is set to W's.  The running means are kept: ugkwp_set_history
 * restores them. */
int ugkwp_set_fields(ugkwp_ctx *ctx, const double *W);
/* The step counter that keys the random numbers (0 <= step < 2^20). */
int ugkwp_set_step(ugkwp_ctx *ctx, int64_t step);
/* Averaging state behind ugkwp_residual and the surface means (host
 * arrays, each may be NULL): per cell the last density, the running sum of
 * the density over the steps and its last running mean [n_cells]; per wall
 * face (all wall faces of a batch, case after case) the last, summed and EMA
 * (p, tau, q) [n_wall*3]; per case
 * {r_inst, r_avg, C_d last, C_d sum, C_d EMA, unused} [n_cases*6].  With
 * ugkwp_set_fields, ugkwp_set_particles and ugkwp_set_step these restore a
 * state taken with the getters exactly (ugkwp_save / ugkwp_load do all of
 * it in one file). */
int ugkwp_get_history(ugkwp_ctx *ctx, double *rho_prev, double *rho_sum, double *rho_mean_prev, double *wlast,
                      double *wsum, double *wema, double *scal);
int ugkwp_set_history(ugkwp_ctx *ctx, const double *rho_prev, const double *rho_sum, const double *rho_mean_prev,
                      const double *wlast, const double *wsum, const double *wema, const double *scal);
/* Checkpoint of the whole committed state to a file: fields, local time
 * steps, the particle store exactly as held on the device, the averaging
 * state, the step counter and the exact-summation windows (the file is
 * written to path.tmp and renamed).  ugkwp_load restores it into a context
 * created with the same mesh and parameters: a run continued from the file
 * gives bit for bit the results of the uninterrupted run (the paper's runs
 * last tens of thousands of steps with averaging windows, Sec. V).  Errors:
 * EIO (file), EINVAL (the file does not match the context), ENOMEM. */
int ugkwp_save(ugkwp_ctx *ctx, const char *path);
int ugkwp_load(ugkwp_ctx *ctx, const char *path);
/* Last committed step's particle tallies sum_k m_k Psi_k before
 * (W^{p,-} Omega) and after (W^{p,+} Omega) transport, Eq. (30),
 * [n_cells*(dim+2)] each. */
int ugkwp_get_tally(ugkwp_ctx *ctx, double *Sminus, double *Splus);
/* Last committed step's time-averaged face fluxes times the face length,
 * F_j s_j (Eqs. (49)-(50)), along each face's normal (outward of its first
 * cell; faces numbered by first appearance over the cells' edges in order),
 * [n_faces*(dim+2)] host; Fs may be NULL to query n_faces; EOVERFLOW if
 * cap < n_faces. */
int ugkwp_get_face_flux(ugkwp_ctx *ctx, double *Fs, int64_t cap, int64_t *n_faces);
/* New particles of the last committed step whose Shakhov
 * acceptance-rejection (Pr != 1) accepted none of its 64 attempts and took
 * the first attempt inside the 6 sqrt(R T^h) cut instead. */
int ugkwp_get_shakhov_fallbacks(ugkwp_ctx *ctx, int64_t *n_capped);

/* Launch tuning (results do not depend on it).  batch_steps: steps enqueued
 * between two host synchronizations (1..1024); use_graph: replay captured
 * HIP graphs of step pairs instead of launching each kernel (not while
 * per-kernel timing is on); transport_block: threads per block of the
 * particle transport (64, 128 or 256); shakhov_lanes: lanes per new
 * particle that evaluate its first Shakhov acceptance-rejection attempts
 * together (1, 2, 4, 8 or 16); max_crossings: face crossings a particle
 * may make in one step before the step fails as a runaway track (ENUMERIC,
 * not committed; 1..10000); scatter_block: threads per block of the
 * re-sort's scatter (its slot claims are per block; 64, 128, 256 or 512);
 * tally_block, flux_block: threads per block of the per-cell tally (one
 * wavefront per cell) and of the face fluxes (one thread per face), each
 * 64, 128 or 256.  ugkwp_get_tuning returns the current values (defaults at
 * init: 32, 1, 256, 4, 10000, 512, 256, 256);
 * ugkwp_set_tuning sets all eight (EINVAL if one is out of range).  None of
 * them changes a result. */
typedef struct {
  int32_t batch_steps, use_graph, transport_block, shakhov_lanes, max_crossings;
  int32_t scatter_block, tally_block, flux_block;
} ugkwp_tuning;
int ugkwp_set_tuning(ugkwp_ctx *ctx, const ugkwp_tuning *t);
int ugkwp_get_tuning(ugkwp_ctx *ctx, ugkwp_tuning *t);

/* Per-kernel timing with HIP events on the library's stream.  enable = 1
 * starts accumulating for every kernel (and resets), 2 for the particle
 * transport kernel only (two events per step, for timing runs), 0 stops.  ugkwp_profile_read returns up
 * to cap entries: name, total milliseconds, launches and the algorithmic
 * bytes moved (the byte model of each kernel). */
int ugkwp_profile(ugkwp_ctx *ctx, int32_t enable);
int ugkwp_profile_read(ugkwp_ctx *ctx, int32_t cap, const char **names, double *ms, int64_t *launches,
                       double *bytes, int32_t *n);

/* Bandwidth reference, outside the step: copies `bytes` bytes from device
 * buffer src to device buffer dst with the library's streaming kernel
 * (16-byte loads and stores, four per thread in flight, grid-stride), once
 * untimed and then `reps` times back to back on `stream` (NULL = the null
 * stream), and stores the mean milliseconds per copy, from HIP events, in
 * *ms_per_copy.  blocks = 0 launches 8 workgroups of 256 threads per compute
 * unit; any other value sets the grid.  Both pointers 16-byte aligned, bytes
 * a positive multiple of 16, regions disjoint, reps >= 1, else UGKWP_EINVAL;
 * a HIP failure gives UGKWP_EDEVICE (no context, so no error text).  It moves
 * 2 * bytes per copy through HBM: the rate the step's kernels are held
 * against beside the datasheet peak. */
int ugkwp_stream_copy(void *dst, const void *src, int64_t bytes, int32_t reps, int32_t blocks, void *stream,
                      double *ms_per_copy);

const char *ugkwp_last_error(const ugkwp_ctx *ctx);
void ugkwp_free(ugkwp_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
