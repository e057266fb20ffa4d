/*
 * CPU oracle for one UGKWP-LTS time step (serial, FP64, plain C).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the package smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or helper with the HIP product library; the two only read the
 * same seeded workloads.
 *
 * Method: Guo, Cao, Long, Xu, "Rigorously justified local time stepping in the
 * unified gas-kinetic wave-particle method" (arXiv 2607.09552), Secs. III-IV:
 *   - local time step from the initial field, Eq. (33), fixed for the run;
 *     global step Eq. (34);
 *   - wave-particle decomposition W = W^h + W^p, Eq. (24), and resampling of
 *     collisionless particles, Eqs. (25)-(26), in the LTS form of Sec. IV.B
 *     (e^{-dt_i/tau_i}, t_f = dt_i);
 *   - free-transport time, Eq. (51);
 *   - transport, Eq. (28), with mass and remaining-time scaling by dt_R/dt_L
 *     at every crossing, Eqs. (41) and (52);
 *   - before/after particle tally, Eqs. (29)-(30);
 *   - time-averaged equilibrium and analytic free-transport wave fluxes,
 *     Eqs. (49)-(50), with the coefficients of Eq. (16) evaluated per side,
 *     Eq. (47), and normalized, Eq. (48);
 *   - conservative update, Eq. (53).
 * Readings where the paper is silent are listed in the repository's design
 * notes and restated at each function below.
 */
#ifndef UGKWP_ORACLE_H
#define UGKWP_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

enum { REF_OK = 0, REF_EINVAL = -1, REF_ENOMEM = -2, REF_EOVERFLOW = -4, REF_ENUMERIC = -5 };
/* REF_BC_WALL_MAXWELL: isothermal wall with accommodation alpha (bface_data
 * T_w, alpha), the boundary condition of the flat-plate case of Sec. V.B: a
 * fraction alpha of what reaches it is re-emitted diffusely, the rest
 * reflected specularly.  A particle hit re-emits diffusely when the fourth
 * uniform of its two WALL draws is below alpha; the wave flux is alpha times
 * the diffuse wall's plus (1 - alpha) times the mirror-state flux. */
enum { REF_BC_FARFIELD = 1, REF_BC_OUTFLOW = 2, REF_BC_WALL = 3, REF_BC_SYMMETRY = 4, REF_BC_WALL_MAXWELL = 6 };

typedef struct {
  int32_t dim;                 /* 1 or 2 */
  int64_t n_nodes;
  const double *nodes;         /* [n_nodes*dim] */
  int64_t n_cells;
  const int64_t *cell_ptr;     /* 2D: CSR of CCW convex polygons; NULL in 1D */
  const int64_t *cell_nodes;
  int64_t n_bfaces;
  const int64_t *bface_nodes;  /* [n_bfaces*dim] */
  const int32_t *bface_type;   /* REF_BC_* */
  const double *bface_data;    /* [n_bfaces*8]: farfield rho,ux,uy,T ; wall T_w */
} ref_mesh;

typedef struct {
  double R, omega, mu_ref, T_ref, Pr;
  int32_t D;                   /* internal degrees of freedom (0..64); particles carry
                                  |xi|^2 / 2 drawn at the local temperature */
  double cfl;
  int32_t n_ref;
  int32_t lts;                 /* 1 local time steps, 0 global (dt_G = min dt_i) */
  uint64_t seed;
  double rho_inf, u_inf_x, u_inf_y, T_inf, L_ref; /* surface coefficients only */
  int32_t wave_only;           /* 1: E = 0 (no particles, all gas in the waves:
                                  the gas-kinetic scheme of the coarse warm-start
                                  solves); 0: UGKWP */
  int32_t dt_source;           /* Eq. (33) reads 0: the initial field, 1: the
                                  freestream (rho_inf, u_inf, T_inf) */
} ref_params;

typedef struct ref_ctx ref_ctx;

int ref_init(const ref_mesh *mesh, const ref_params *par, const double *W0, ref_ctx **out);
int ref_step(ref_ctx *c, int32_t n_steps);
int ref_get_fields(const ref_ctx *c, double *W);
int ref_set_fields(ref_ctx *c, const double *W);
int ref_get_dt(const ref_ctx *c, double *dt);
int ref_get_counts(const ref_ctx *c, int32_t *count, int64_t *n_total, int64_t *n_new,
                   int64_t *n_removed, int64_t *n_exited);
/* ei: internal energy per unit mass |xi|^2 / 2 of each particle (D > 0);
   may be NULL (read: skipped; write: 0) */
int ref_get_particles(const ref_ctx *c, int64_t cap, uint64_t *pid, int32_t *cell, double *m,
                      double *x, double *u, double *ei, int64_t *n);
int ref_set_particles(ref_ctx *c, int64_t n, const uint64_t *pid, const int32_t *cell,
                      const double *m, const double *x, const double *u, const double *ei);
int ref_residual(const ref_ctx *c, double *r_inst, double *r_avg, int64_t *step);
int ref_surface(const ref_ctx *c, int32_t mode, double *out, int64_t cap, int64_t *n_wall,
                double *Cd);
int ref_get_tally(const ref_ctx *c, double *Sminus, double *Splus); /* last step, [nc*(dim+2)] */
int ref_get_face_flux(const ref_ctx *c, double *Fs);               /* last step, [nf*(dim+2)] */
int64_t ref_n_faces(const ref_ctx *c);
int64_t ref_n_guard(const ref_ctx *c); /* cells reset by the vacuum guard in the last step */
void ref_set_step(ref_ctx *c, int64_t step); /* step counter that keys the RNG */
const char *ref_last_error(const ref_ctx *c);
void ref_free(ref_ctx *c);

/* ---- stage-level entry points used by the pins ---- */
void ref_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double ref_uniform(uint32_t a, uint32_t b);
/* out = {abar, bbar, cbar, dbar, ebar, E, dbar - E, ebar + dt E / 2} for (dt, tau) */
void ref_time_coeffs(double dt, double tau, double out[8]);
/* half-range (sign +1/-1) or full (0) moments <u^k>, k = 0..6, of a unit-density
   1D Maxwellian with mean U and lambda = 1/(2RT) */
void ref_moments_n(double U, double lam, int sign, double M[7]);
/* microslope (a0, an, at, a4) of the Maxwellian of W (face frame, 4 comps)
   for the normal derivative dW, with lambda' divided by Pr */
void ref_microslope(const double W[4], const double dW[4], int K, double Pr, double a[4]);
/* interior face flux in the face frame (per unit length, time averaged) */
void ref_flux_interior(const double WL[4], const double WR[4], const double dW0[4],
                       const double *WhL, const double *WhR, const double dWhL[4],
                       const double dWhR[4], double dtL, double tauL, double dtR, double tauR,
                       int K, double Pr, int wave_only, double Feq[4], double Ffr[4]);
/* diffuse-wall face flux (face frame, normal out of the gas) */
void ref_flux_wall(const double W[4], const double *Wh, double dt, double tau, double Tw, double R,
                   int K, int wave_only, double F[4]);
/* wave_only: the free-transport wave carries all of g^h (coefficients dbar,
   ebar instead of dbar - E, ebar + dt E / 2): no particles take a share */
/* track one particle through the mesh of c for remaining time t, no RNG at
   symmetry faces; diffuse walls draw with (pid, step).  Returns 0 if it ends
   inside (cell_out), 1 if it left through a far-field/outflow face. */
int ref_track_one(ref_ctx *c, uint64_t pid, int64_t step, int32_t cell, double x[2], double u[3],
                  double *m, double t, int32_t *cell_out, int32_t *n_cross);
/* exactly rounded sum of x[0..n) (nearest, ties to even) */
double ref_exact_sum(const double *x, int64_t n);
/* reconstruction of one side of a face (Wfar NULL: first order) and the face
   values/slopes of interior face fi from the current fields (face frame) */
void ref_reconstruct(const double *Wfar, double xfar, const double Wself[4], double xself, const double Wother[4],
                     double xother, int K, double out[4], double slope[4]);
int ref_face_geom(const ref_ctx *c, int64_t fi, double out[8]);
int ref_face_values(const ref_ctx *c, int64_t fi, double WLf[4], double WRf[4], double sl[4], double sr[4],
                    double dW0[4]);
/* vacuum guard on an updated state Wn [dim + 2] of a cell of volume vol with
   post-transport particle tally Sp [dim + 2]; returns 1 if Wn was replaced */
int ref_vacuum_guard(const ref_ctx *c, const double *Sp, double vol, double *Wn);
/* deviation z of a new particle (Maxwellian, or Shakhov acceptance-rejection
   when shak = {U_x, U_y, T, p, Q_x, Q_y} is given); returns 1 when no attempt
   was accepted (then z is the first attempt within c_max, or 0) */
int ref_sample_deviation(ref_ctx *c, uint64_t pid, int64_t step, const double Uh[2], double Th, const double *shak,
                         double z[3]);
/* Shakhov draws of the last step that took the 64-attempt fallback */
int64_t ref_n_capped(const ref_ctx *c);
/* averaging state (restart): rho_prev, rho_sum, rho_mean_prev [nc]; wall
   faces' last, summed and EMA (p, tau, q) [nwall*3]; C_d last, sum, EMA */
int ref_get_history(const ref_ctx *c, double *rho_prev, double *rho_sum, double *rho_mean_prev, double *wlast,
                    double *wsum, double *wema, double cd[3]);
int ref_set_history(ref_ctx *c, const double *rho_prev, const double *rho_sum, const double *rho_mean_prev,
                    const double *wlast, const double *wsum, const double *wema, const double cd[3]);

#ifdef __cplusplus
}
#endif
#endif
