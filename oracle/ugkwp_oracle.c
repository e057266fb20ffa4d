/*
 * CPU oracle for one UGKWP-LTS time step.  TEST INFRASTRUCTURE ONLY: only the
 * tests, the package smoke check and the benchmark's CPU-baseline leg may load
 * it.  Plain serial C, FP64 throughout, built with -O2 -ffp-contract=off.
 *
 * Every step follows the paper (arXiv 2607.09552) in its own order and
 * notation; the cited equation numbers are the paper's.  Where the paper is
 * silent the reading used is stated at the function.  Pins: the
 * reconstruction (MUSCL, van Leer) and the equilibrium slope by exactness on
 * linear fields over graded meshes, the positivity guard branch by branch,
 * the whole step by an independent literal GTS step (equal time steps), the
 * collisionless limit by free-molecular wall fluxes on a plate, the Shakhov
 * acceptance-rejection, the diffuse wall's re-emission and the far-field
 * ghost slab statistically by the distributions and fluxes they must give,
 * the upwind g0^h of Eq. (50) by the collisionless transport of the
 * piecewise initial reconstruction, integrated by quadrature in t and u.
 */
#include "ugkwp_oracle.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define MAXV 8          /* max polygon vertices */
#define MAX_CROSS 10000 /* crossings per particle and step before ENUMERIC */

/* particle flags */
#define F_COLLIDE 1
#define F_GHOST 2
#define F_NEW 4
#define F_EXIT 8

/* RNG purposes (counter word 3 = purpose << 24 | call) */
#define P_FREE 0u
#define P_POS 1u
#define P_VEL 2u
#define P_WALL 3u

static int is_wall(int32_t ty) { return ty == REF_BC_WALL || ty == REF_BC_WALL_MAXWELL; }
#define P_SHAKHOV 4u
#define P_INTERNAL 5u
/* wall hit h of a particle draws its internal energy from INTERNAL calls
 * WALL_INTERNAL_CALL0 + h ceil(D/2) + j; birth uses calls j */
#define WALL_INTERNAL_CALL0 256u

/* accumulator of an exactly rounded sum (see xs_add) */
typedef struct {
  int n, cap;
  double *p;      /* partials, increasing magnitude */
  double inl[6];  /* inline storage for the first partials */
  int nonfinite;  /* a term was inf or nan: the result is their plain sum */
  double naive;
} xsum;

static const double TWO_PI = 6.283185307179586;
static const double PI = 3.141592653589793;

typedef struct {
  uint64_t pid;
  int32_t cell;  /* current cell (interior id) */
  int32_t flags;
  double x[2], u[3], m, t; /* t: remaining free-transport time */
  double ei;                /* internal energy per unit mass, |xi|^2 / 2 (0 when D = 0) */
} particle;

struct ref_ctx {
  int dim, nw, K, N; /* nw = dim + 2 stored components; K lumped dofs in the face frame; N = K + 2 */
  ref_params p;
  int64_t nc, nn, nb, nf;
  double *nodes;
  /* cells */
  int64_t *cptr;   /* local face CSR [nc+1] */
  int64_t *cvtx;   /* vertex id of local face k (its start vertex) */
  double *vol, *cen;
  double *lfn;     /* per local face: nx, ny, c (= n . v_start), s */
  int64_t *lnb;    /* per local face: neighbour cell, or -(b+1) for boundary face b */
  int64_t *lface;  /* per local face: global face id */
  /* faces */
  int64_t *fL, *fR, *fkL, *fkR; /* fR = -(b+1) on boundary; fk*: local face index in the cell */
  double *fn, *fs, *fmid;
  /* boundary faces */
  int64_t *bcell, *bk;
  int32_t *btype;
  double *bdata;
  /* state */
  double *W, *dt, *ratio; /* ratio per local face: dt_neighbour / dt_self (1 on boundary) */
  double *rho_prev, *rho_sum, *rho_mean_prev;
  particle *P;
  int64_t np, cap;
  int64_t step;
  double r_inst, r_avg;
  /* last-step diagnostics */
  double *Sm, *Sp, *Fs;
  int32_t *count;
  int64_t n_total, n_new, n_removed, n_exited, n_guard;
  /* surface */
  int64_t nwall;
  int64_t *wall_b;                 /* boundary face id of each wall face */
  double *wimp;                    /* per boundary face: particle impulse x,y and energy */
  xsum *xwimp;                     /* their exact sums during a step */
  int64_t n_capped;                /* Shakhov draws that took the 64-attempt fallback (last step) */
  double *wsurf_last, *wsurf_sum, *wsurf_ema; /* per wall face: p, tau, q */
  double cd_last, cd_sum, cd_ema;
  char err[256];
};

static int fail(ref_ctx *c, int code, const char *fmt, ...) {
  if (c) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(c->err, sizeof c->err, fmt, ap);
    va_end(ap);
  }
  return code;
}

/* ======================================================================== */
/* Exactly rounded sums                                                      */
/* ======================================================================== */

/* The tallies of Eqs. (24), (29)-(30) and the other sums over particles are
 * plain sums; the oracle takes the FP64 value nearest to the exact sum (ties
 * to even), so that the result does not depend on the order of the terms.
 * Method: Shewchuk, "Adaptive precision floating-point arithmetic and fast
 * robust geometric predicates" (1997): the running sum is kept exactly as a
 * list of nonoverlapping partials of increasing magnitude, each new term is
 * merged by error-free two-sums; the final rounding adds the partials from
 * the top and settles an exact half-way case by the sign of the next
 * partial below. */

static void xs_init(xsum *s) {
  s->n = 0;
  s->cap = 6;
  s->p = s->inl;
  s->nonfinite = 0;
  s->naive = 0.0;
}

static void xs_free(xsum *s) {
  if (s->p != s->inl) free(s->p);
  xs_init(s);
}

static void xs_add(xsum *s, double x) {
  if (!isfinite(x) || s->nonfinite) {
    if (!s->nonfinite) {
      s->naive = 0.0;
      for (int j = 0; j < s->n; ++j) s->naive += s->p[j];
    }
    s->nonfinite = 1;
    s->naive += x;
    return;
  }
  int i = 0;
  for (int j = 0; j < s->n; ++j) {
    double y = s->p[j];
    if (fabs(x) < fabs(y)) {
      double t = x;
      x = y;
      y = t;
    }
    double hi = x + y;
    double lo = y - (hi - x);
    if (lo != 0.0) s->p[i++] = lo;
    x = hi;
  }
  if (i == s->cap) {
    int ncap = 2 * s->cap;
    double *q = malloc(sizeof(double) * (size_t)ncap);
    if (!q) abort();
    memcpy(q, s->p, sizeof(double) * (size_t)i);
    if (s->p != s->inl) free(s->p);
    s->p = q;
    s->cap = ncap;
  }
  s->p[i++] = x;
  s->n = i;
}

static double xs_round(const xsum *s) {
  if (s->nonfinite) return s->naive;
  int n = s->n;
  if (n == 0) return 0.0;
  double hi = s->p[--n], lo = 0.0;
  while (n > 0) {
    double x = hi, y = s->p[--n];
    hi = x + y;
    double yr = hi - x;
    lo = y - yr;
    if (lo != 0.0) break;
  }
  if (n > 0 && ((lo < 0.0 && s->p[n - 1] < 0.0) || (lo > 0.0 && s->p[n - 1] > 0.0))) {
    double y = lo * 2.0;
    double x = hi + y;
    double yr = x - hi;
    if (y == yr) hi = x;
  }
  return hi;
}

/* n accumulators in one block */
static xsum *xs_array(int64_t n) {
  xsum *a = calloc((size_t)(n ? n : 1), sizeof(xsum));
  if (!a) abort();
  for (int64_t k = 0; k < n; ++k) xs_init(&a[k]);
  return a;
}

static void xs_array_free(xsum *a, int64_t n) {
  for (int64_t k = 0; k < n; ++k) xs_free(&a[k]);
  free(a);
}

double ref_exact_sum(const double *x, int64_t n) {
  xsum s;
  xs_init(&s);
  for (int64_t k = 0; k < n; ++k) xs_add(&s, x[k]);
  double r = xs_round(&s);
  xs_free(&s);
  return r;
}

/* ======================================================================== */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), from its definition.  */
/* ======================================================================== */

void ref_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

/* 52 random bits -> (k + 1/2) 2^-52, exact in FP64, strictly inside (0,1). */
double ref_uniform(uint32_t a, uint32_t b) {
  uint64_t k = ((uint64_t)a << 20) | (uint64_t)(b >> 12);
  return ((double)k + 0.5) * 2.220446049250313e-16;
}

/* Two uniforms from counter (pid, step, purpose, call) under key = seed. */
static void draw2(uint64_t seed, uint64_t pid, int64_t step, uint32_t purpose, uint32_t call,
                  double *e0, double *e1) {
  uint32_t ctr[4] = {(uint32_t)pid, (uint32_t)(pid >> 32), (uint32_t)step, (purpose << 24) | call};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t o[4];
  ref_philox4x32_10(ctr, key, o);
  *e0 = ref_uniform(o[0], o[1]);
  *e1 = ref_uniform(o[2], o[3]);
}

/* Box-Muller pair from two uniforms. */
static void box_muller(double e0, double e1, double *z0, double *z1) {
  double r = sqrt(-2.0 * log(e0));
  double a = TWO_PI * e1;
  *z0 = r * cos(a);
  *z1 = r * sin(a);
}

/* ======================================================================== */
/* Time-integration coefficients, Eq. (16), normalized per side, Eq. (48).   */
/* ======================================================================== */

/* With x = dt/tau, E = e^{-x} and phi = (1 - E)/x, Eq. (16) divided by dt is
 *   abar = 1 - phi,              bbar = tau (2 phi - 1 - E),
 *   cbar = tau (x/2 - 1 + phi),  dbar = phi,            ebar = tau (E - phi).
 * The free-transport wave flux, Eq. (50), uses dbar - E and ebar + dt E / 2.
 * For x < 1 every difference is summed from its Taylor series in x (terms
 * (-x)^k/(k+1)!), since the closed forms cancel catastrophically for small x.
 */
void ref_time_coeffs(double dt, double tau, double out[8]) {
  double x = dt / tau;
  double E = exp(-x);
  double phi, a, b, cc, e, dmE, g;
  if (x < 1.0) {
    enum { KMAX = 30 };
    double t[KMAX + 1];
    t[0] = 1.0;
    for (int k = 1; k <= KMAX; ++k) t[k] = t[k - 1] * (-x) / (double)(k + 1);
    double s_phi = 0.0, s_a = 0.0, s_c = 0.0, s_b = 0.0, s_e = 0.0, s_g = 0.0;
    for (int k = KMAX; k >= 0; --k) {
      s_phi += t[k];
      if (k >= 1) {
        s_a += t[k];
        s_e += (double)k * t[k];
      }
      if (k >= 2) {
        s_c += t[k];
        s_b += (double)(1 - k) * t[k];
        s_g += 0.5 * (double)(k * (1 - k)) * t[k];
      }
    }
    phi = s_phi;
    a = -s_a;
    cc = s_c;
    b = s_b;
    e = s_e;
    dmE = -s_e;
    g = s_g;
  } else {
    phi = (1.0 - E) / x;
    a = 1.0 - phi;
    b = (2.0 * phi - 1.0) - E;
    cc = (0.5 * x - 1.0) + phi;
    e = E - phi;
    dmE = phi - E;
    g = (E - phi) + 0.5 * x * E;
  }
  out[0] = a;
  out[1] = tau * b;
  out[2] = tau * cc;
  out[3] = phi;
  out[4] = tau * e;
  out[5] = E;
  out[6] = dmE;
  out[7] = tau * g;
}

/* ======================================================================== */
/* Moments of the Maxwellian, Eq. (1), in the face frame.                    */
/* ======================================================================== */

/* <u^k>, k = 0..6, over u > 0 (sign +1), u < 0 (sign -1) or all u (0), for a
 * unit-density normal Maxwellian with mean U and lambda = 1/(2RT).  Half-range
 * start values from erfc; higher moments by the recursion
 * M_{k+2} = U M_{k+1} + (k+1)/(2 lambda) M_k (integration by parts). */
void ref_moments_n(double U, double lam, int sign, double M[7]) {
  if (sign == 0) {
    M[0] = 1.0;
    M[1] = U;
  } else {
    double sl = sqrt(lam);
    double ex = exp(-lam * U * U) / (2.0 * sqrt(PI * lam));
    if (sign > 0) {
      M[0] = 0.5 * erfc(-sl * U);
      M[1] = U * M[0] + ex;
    } else {
      M[0] = 0.5 * erfc(sl * U);
      M[1] = U * M[0] - ex;
    }
  }
  for (int k = 0; k + 2 <= 6; ++k) M[k + 2] = U * M[k + 1] + (double)(k + 1) / (2.0 * lam) * M[k];
}

typedef struct {
  double Mn[7], Mt[5], X[3];
} moments;

/* tangential <v^k> (k = 0..4, full range) and lumped <xi^{2d}> (d = 0..2). */
static void set_moments(moments *m, double U, double V, double lam, int K, int sign) {
  ref_moments_n(U, lam, sign, m->Mn);
  m->Mt[0] = 1.0;
  m->Mt[1] = V;
  for (int k = 0; k + 2 <= 4; ++k) m->Mt[k + 2] = V * m->Mt[k + 1] + (double)(k + 1) / (2.0 * lam) * m->Mt[k];
  m->X[0] = 1.0;
  m->X[1] = (double)K / (2.0 * lam);
  m->X[2] = (double)(K * (K + 2)) / (4.0 * lam * lam);
}

static double mom(const moments *m, int a, int b, int d) { return m->Mn[a] * m->Mt[b] * m->X[d]; }

/* <u_n^a u_t^b xi^{2d} Psi>, Psi = (1, u_n, u_t, (u_n^2 + u_t^2 + xi^2)/2), Eq. (6). */
static void psi_mom(const moments *m, int a, int b, int d, double out[4]) {
  out[0] = mom(m, a, b, d);
  out[1] = mom(m, a + 1, b, d);
  out[2] = mom(m, a, b + 1, d);
  out[3] = 0.5 * (mom(m, a + 2, b, d) + mom(m, a, b + 2, d) + mom(m, a, b, d + 1));
}

/* <u_n^a Psi phi> with phi = c0 + cn u_n + ct u_t + c4 (u_n^2 + u_t^2 + xi^2)/2,
 * the expansion of Eqs. (19) and (21). */
static void psi_poly(const moments *m, int a, const double c[4], double out[4]) {
  double t0[4], t1[4], t2[4], t3[4], t4[4], t5[4];
  psi_mom(m, a, 0, 0, t0);
  psi_mom(m, a + 1, 0, 0, t1);
  psi_mom(m, a, 1, 0, t2);
  psi_mom(m, a + 2, 0, 0, t3);
  psi_mom(m, a, 2, 0, t4);
  psi_mom(m, a, 0, 1, t5);
  for (int q = 0; q < 4; ++q)
    out[q] = c[0] * t0[q] + c[1] * t1[q] + c[2] * t2[q] + c[3] * (0.5 * (t3[q] + t4[q] + t5[q]));
}

/* Face-frame primitive state of W = (rho, rho U, rho V, rho E):
 * lambda = N rho / (4 e) with e = rho E - rho (U^2 + V^2)/2 and N = K + 2. */
typedef struct {
  double rho, U, V, lam;
} fstate;

static fstate face_state(const double W[4], int K) {
  fstate s;
  s.rho = W[0];
  s.U = W[1] / W[0];
  s.V = W[2] / W[0];
  double e = W[3] - 0.5 * s.rho * (s.U * s.U + s.V * s.V);
  s.lam = ((double)(K + 2) * s.rho) / (4.0 * e);
  return s;
}

/* Microslope of ln g, Eqs. (18)-(20): the derivative of the Maxwellian of W
 * along the face normal for the conservative derivative dW, expanded as in
 * Eq. (19).  Prandtl correction (Sec. III.A): lambda' is divided by Pr before
 * the coefficients are formed; Pr = 1 solves Eq. (20) exactly. */
void ref_microslope(const double W[4], const double dW[4], int K, double Pr, double a[4]) {
  fstate s = face_state(W, K);
  double N = (double)(K + 2);
  double rho = s.rho, U = s.U, V = s.V, lam = s.lam;
  double dU = (dW[1] - U * dW[0]) / rho;
  double dV = (dW[2] - V * dW[0]) / rho;
  double e = W[3] - 0.5 * rho * (U * U + V * V);
  double de = (dW[3] - 0.5 * dW[0] * (U * U + V * V)) - rho * (U * dU + V * dV);
  double dlam = N * (dW[0] * e - rho * de) / (4.0 * e * e);
  dlam = dlam / Pr;
  a[3] = -2.0 * dlam;
  a[1] = 2.0 * (dlam * U + lam * dU);
  a[2] = 2.0 * (dlam * V + lam * dV);
  a[0] = ((dW[0] / rho + 0.5 * N * (dlam / lam)) - dlam * (U * U + V * V)) - 2.0 * lam * (U * dU + V * dV);
}

/* Interior face, face frame (normal n from L to R, tangent t = (-n_y, n_x)).
 *   W0 from the half-range moments of g_L, g_R, Eq. (17);
 *   a from the slope dW0 (one continuous normal slope, tangential derivatives
 *   neglected) with the Prandtl fix, A from the compatibility relation Eq. (22);
 *   Feq: Eq. (49) with per-side normalized coefficients, Eqs. (47)-(48);
 *   Ffr: Eq. (50); g0^h read upwind (u_n > 0 from the left hydrodynamic state
 *   and its slope, u_n < 0 from the right).  A side whose W^h is not a valid
 *   Maxwellian (WhL / WhR NULL) contributes no free-transport wave flux. */
void ref_flux_interior(const double WL[4], const double WR[4], const double dW0[4],
                       const double *WhL, const double *WhR, const double dWhL[4],
                       const double dWhR[4], double dtL, double tauL, double dtR, double tauR,
                       int K, double Pr, int wave_only, double Feq[4], double Ffr[4]) {
  fstate sL = face_state(WL, K), sR = face_state(WR, K);
  moments mL, mR;
  set_moments(&mL, sL.U, sL.V, sL.lam, K, +1);
  set_moments(&mR, sR.U, sR.V, sR.lam, K, -1);
  double pL[4], pR[4], W0[4];
  psi_mom(&mL, 0, 0, 0, pL);
  psi_mom(&mR, 0, 0, 0, pR);
  for (int q = 0; q < 4; ++q) W0[q] = sL.rho * pL[q] + sR.rho * pR[q];
  fstate s0 = face_state(W0, K);
  double cL[8], cR[8];
  ref_time_coeffs(dtL, tauL, cL);
  ref_time_coeffs(dtR, tauR, cR);
  if (wave_only) {
    cL[6] = cL[3];
    cL[7] = cL[4];
    cR[6] = cR[3];
    cR[7] = cR[4];
  }
  /* Reading (the paper does not meet the case): when both sides move away
   * from the face so fast that the interface holds no gas in FP64 -- W0's
   * density below 1e-30 of the two sides' or not a valid Maxwellian, as for
   * a cell leaving a wall or a symmetry face at high Mach number -- there is
   * no equilibrium flux; likewise if the flux itself is not finite. */
  if (!(W0[0] > 1e-30 * (sL.rho + sR.rho)) || !(s0.lam > 0.0) || !(s0.lam < HUGE_VAL)) {
    for (int q = 0; q < 4; ++q) Feq[q] = 0.0;
  } else {
    double a[4], A[4], Wt[4], tmp[4];
    ref_microslope(W0, dW0, K, Pr, a);
    moments m0f, m0p, m0m;
    set_moments(&m0f, s0.U, s0.V, s0.lam, K, 0);
    set_moments(&m0p, s0.U, s0.V, s0.lam, K, +1);
    set_moments(&m0m, s0.U, s0.V, s0.lam, K, -1);
    psi_poly(&m0f, 1, a, tmp);
    for (int q = 0; q < 4; ++q) Wt[q] = -s0.rho * tmp[q];
    ref_microslope(W0, Wt, K, 1.0, A);
    double f1p[4], fap[4], fAp[4], f1m[4], fam[4], fAm[4];
    psi_mom(&m0p, 1, 0, 0, f1p);
    psi_poly(&m0p, 2, a, fap);
    psi_poly(&m0p, 1, A, fAp);
    psi_mom(&m0m, 1, 0, 0, f1m);
    psi_poly(&m0m, 2, a, fam);
    psi_poly(&m0m, 1, A, fAm);
    for (int q = 0; q < 4; ++q)
      Feq[q] = s0.rho * ((cL[0] * f1p[q] + cL[1] * fap[q]) + cL[2] * fAp[q]) +
               s0.rho * ((cR[0] * f1m[q] + cR[1] * fam[q]) + cR[2] * fAm[q]);
    if (!isfinite(Feq[0]) || !isfinite(Feq[1]) || !isfinite(Feq[2]) || !isfinite(Feq[3]))
      for (int q = 0; q < 4; ++q) Feq[q] = 0.0;
  }

  for (int q = 0; q < 4; ++q) Ffr[q] = 0.0;
  if (WhL) {
    fstate h = face_state(WhL, K);
    double ah[4], g1[4], ga[4];
    ref_microslope(WhL, dWhL, K, 1.0, ah);
    moments mh;
    set_moments(&mh, h.U, h.V, h.lam, K, +1);
    psi_mom(&mh, 1, 0, 0, g1);
    psi_poly(&mh, 2, ah, ga);
    for (int q = 0; q < 4; ++q) Ffr[q] += h.rho * (cL[6] * g1[q] + cL[7] * ga[q]);
  }
  if (WhR) {
    fstate h = face_state(WhR, K);
    double ah[4], g1[4], ga[4];
    ref_microslope(WhR, dWhR, K, 1.0, ah);
    moments mh;
    set_moments(&mh, h.U, h.V, h.lam, K, -1);
    psi_mom(&mh, 1, 0, 0, g1);
    psi_poly(&mh, 2, ah, ga);
    for (int q = 0; q < 4; ++q) Ffr[q] += h.rho * (cR[6] * g1[q] + cR[7] * ga[q]);
  }
}

/* Diffuse isothermal wall (the paper states only "diffuse reflection" and
 * that both half-space fluxes use dt_i at a physical boundary).  Reading:
 * first order, the outgoing half (u_n > 0, into the wall) carries
 * abar g(W_i) + (dbar - E) g(W^h_i); the reflected half is a wall Maxwellian
 * at rest and T_w whose density makes the net wave mass flux zero. */
void ref_flux_wall(const double W[4], const double *Wh, double dt, double tau, double Tw, double R,
                   int K, int wave_only, double F[4]) {
  double co[8], t[4];
  ref_time_coeffs(dt, tau, co);
  if (wave_only) {
    co[6] = co[3];
    co[7] = co[4];
  }
  fstate s = face_state(W, K);
  moments m;
  set_moments(&m, s.U, s.V, s.lam, K, +1);
  psi_mom(&m, 1, 0, 0, t);
  for (int q = 0; q < 4; ++q) F[q] = s.rho * co[0] * t[q];
  if (Wh) {
    fstate h = face_state(Wh, K);
    set_moments(&m, h.U, h.V, h.lam, K, +1);
    psi_mom(&m, 1, 0, 0, t);
    for (int q = 0; q < 4; ++q) F[q] += h.rho * co[6] * t[q];
  }
  double lw = 1.0 / (2.0 * R * Tw);
  moments mw;
  set_moments(&mw, 0.0, 0.0, lw, K, -1);
  psi_mom(&mw, 1, 0, 0, t);
  double rw = F[0] / (-t[0]);
  for (int q = 0; q < 4; ++q) F[q] += rw * t[q];
}

/* ======================================================================== */
/* Gas relations                                                             */
/* ======================================================================== */

typedef struct {
  double rho, ux, uy, T, e;
} prim_t;

/* primitive variables of a stored W (dim + 2 comps); e = rho E - rho |U|^2/2,
 * T = 2 e / (N R rho) with N = 3 + D velocity-like degrees of freedom. */
static prim_t prim(const ref_ctx *c, const double *W) {
  prim_t s;
  s.rho = W[0];
  s.ux = W[1] / s.rho;
  s.uy = c->dim == 2 ? W[2] / s.rho : 0.0;
  double ke = 0.5 * s.rho * (s.ux * s.ux + s.uy * s.uy);
  s.e = W[c->dim + 1] - ke;
  s.T = (2.0 * s.e) / ((double)c->N * c->p.R * s.rho);
  return s;
}

static int prim_ok(prim_t s) { return s.rho > 0.0 && s.e > 0.0 && isfinite(s.rho) && isfinite(s.e); }

/* tau = mu / p, Eq. (3), with mu = mu_ref (T/T_ref)^omega (VHS). */
static double relax_time(const ref_ctx *c, double rho, double T) {
  double mu = c->p.mu_ref * pow(T / c->p.T_ref, c->p.omega);
  return mu / (rho * c->p.R * T);
}

/* stored W (dim + 2) -> face frame (rho, rho U.n, rho U.t, rho E), t = (-n_y, n_x) */
static void to_frame(const ref_ctx *c, const double *W, const double n[2], double out[4]) {
  out[0] = W[0];
  if (c->dim == 2) {
    out[1] = W[1] * n[0] + W[2] * n[1];
    out[2] = W[2] * n[0] - W[1] * n[1];
    out[3] = W[3];
  } else {
    out[1] = W[1] * n[0];
    out[2] = 0.0;
    out[3] = W[2];
  }
}

static void from_frame(const ref_ctx *c, const double F[4], const double n[2], double *out) {
  out[0] = F[0];
  if (c->dim == 2) {
    out[1] = F[1] * n[0] - F[2] * n[1];
    out[2] = F[1] * n[1] + F[2] * n[0];
    out[3] = F[3];
  } else {
    out[1] = F[1] * n[0];
    out[2] = F[3];
  }
}

/* ======================================================================== */
/* Mesh                                                                      */
/* ======================================================================== */

typedef struct {
  int64_t a, b, cell, k;
} edge_t;

static int edge_cmp(const void *x, const void *y) {
  const edge_t *p = x, *q = y;
  if (p->a != q->a) return p->a < q->a ? -1 : 1;
  if (p->b != q->b) return p->b < q->b ? -1 : 1;
  if (p->cell != q->cell) return p->cell < q->cell ? -1 : 1;
  return p->k < q->k ? -1 : (p->k > q->k);
}

static void *xcalloc(size_t n, size_t s) { return calloc(n ? n : 1, s); }

/* Cell geometry by fan triangulation from vertex 0: area (Omega_i),
 * centroid, per-edge outward unit normal n = (dy, -dx)/|d| of the CCW edge
 * d = v_{k+1} - v_k, its length s_j and offset n . v_k. */
static int build_mesh(ref_ctx *c, const ref_mesh *m) {
  int64_t nc = m->n_cells, nb = m->n_bfaces;
  c->nc = nc;
  c->nb = nb;
  c->nn = m->n_nodes;
  c->nodes = xcalloc((size_t)(m->n_nodes * c->dim), sizeof(double));
  memcpy(c->nodes, m->nodes, sizeof(double) * (size_t)(m->n_nodes * c->dim));
  c->cptr = xcalloc((size_t)nc + 1, sizeof(int64_t));
  if (c->dim == 1) {
    for (int64_t i = 0; i <= nc; ++i) c->cptr[i] = 2 * i;
  } else {
    for (int64_t i = 0; i <= nc; ++i) c->cptr[i] = m->cell_ptr[i];
    for (int64_t i = 0; i < nc; ++i) {
      int64_t nv = c->cptr[i + 1] - c->cptr[i];
      if (nv < 3 || nv > MAXV) return fail(c, REF_EINVAL, "cell %lld has %lld vertices", (long long)i, (long long)nv);
    }
  }
  int64_t nl = c->cptr[nc];
  c->cvtx = xcalloc((size_t)nl, sizeof(int64_t));
  c->lfn = xcalloc((size_t)nl * 4, sizeof(double));
  c->lnb = xcalloc((size_t)nl, sizeof(int64_t));
  c->lface = xcalloc((size_t)nl, sizeof(int64_t));
  c->vol = xcalloc((size_t)nc, sizeof(double));
  c->cen = xcalloc((size_t)nc * 2, sizeof(double));
  c->bcell = xcalloc((size_t)nb, sizeof(int64_t));
  c->bk = xcalloc((size_t)nb, sizeof(int64_t));
  c->btype = xcalloc((size_t)nb, sizeof(int32_t));
  c->bdata = xcalloc((size_t)nb * 8, sizeof(double));
  for (int64_t b = 0; b < nb; ++b) c->bcell[b] = -1;
  memcpy(c->btype, m->bface_type, sizeof(int32_t) * (size_t)nb);
  memcpy(c->bdata, m->bface_data, sizeof(double) * (size_t)nb * 8);
  for (int64_t b = 0; b < nb; ++b)
    if ((c->btype[b] < REF_BC_FARFIELD || c->btype[b] > REF_BC_SYMMETRY) && c->btype[b] != REF_BC_WALL_MAXWELL)
      return fail(c, REF_EINVAL, "boundary face %lld has unknown type %d", (long long)b, c->btype[b]);

  if (c->dim == 1) {
    const double *x = c->nodes;
    for (int64_t i = 0; i < nc; ++i) {
      if (!(x[i + 1] > x[i])) return fail(c, REF_EINVAL, "1D nodes not increasing at %lld", (long long)i);
      c->vol[i] = x[i + 1] - x[i];
      c->cen[2 * i] = 0.5 * (x[i] + x[i + 1]);
      c->cvtx[2 * i] = i;
      c->cvtx[2 * i + 1] = i + 1;
      double *f0 = c->lfn + 8 * i, *f1 = f0 + 4;
      f0[0] = -1.0; f0[1] = 0.0; f0[2] = -x[i]; f0[3] = 1.0;
      f1[0] = 1.0; f1[1] = 0.0; f1[2] = x[i + 1]; f1[3] = 1.0;
      c->lnb[2 * i] = i - 1;
      c->lnb[2 * i + 1] = i + 1;
    }
    int64_t seen[2] = {0, 0};
    for (int64_t b = 0; b < nb; ++b) {
      int64_t nd = m->bface_nodes[b];
      if (nd == 0) {
        c->lnb[0] = -(b + 1); c->bcell[b] = 0; c->bk[b] = 0; seen[0]++;
      } else if (nd == nc) {
        c->lnb[2 * (nc - 1) + 1] = -(b + 1); c->bcell[b] = nc - 1; c->bk[b] = 1; seen[1]++;
      } else {
        return fail(c, REF_EINVAL, "1D boundary face on interior node %lld", (long long)nd);
      }
    }
    if (seen[0] != 1 || seen[1] != 1) return fail(c, REF_EINVAL, "1D mesh needs one boundary face at each end");
  } else {
    const double *v = c->nodes;
    for (int64_t i = 0; i < nc; ++i) {
      int64_t s0 = c->cptr[i], nv = c->cptr[i + 1] - s0;
      const int64_t *id = m->cell_nodes + s0;
      for (int64_t k = 0; k < nv; ++k)
        if (id[k] < 0 || id[k] >= m->n_nodes) return fail(c, REF_EINVAL, "cell %lld node out of range", (long long)i);
      double x0 = v[2 * id[0]], y0 = v[2 * id[0] + 1];
      double area = 0.0, cx = 0.0, cy = 0.0;
      for (int64_t t = 0; t + 2 < nv; ++t) {
        double xa = v[2 * id[t + 1]], ya = v[2 * id[t + 1] + 1];
        double xb = v[2 * id[t + 2]], yb = v[2 * id[t + 2] + 1];
        double At = 0.5 * ((xa - x0) * (yb - y0) - (xb - x0) * (ya - y0));
        area += At;
        cx += At * ((x0 + xa + xb) / 3.0);
        cy += At * ((y0 + ya + yb) / 3.0);
      }
      if (!(area > 0.0)) return fail(c, REF_EINVAL, "cell %lld has non-positive area (not CCW?)", (long long)i);
      c->vol[i] = area;
      c->cen[2 * i] = cx / area;
      c->cen[2 * i + 1] = cy / area;
      for (int64_t k = 0; k < nv; ++k) {
        int64_t a = id[k], b = id[(k + 1) % nv], bb = id[(k + 2) % nv];
        double dx = v[2 * b] - v[2 * a], dy = v[2 * b + 1] - v[2 * a + 1];
        double ex = v[2 * bb] - v[2 * b], ey = v[2 * bb + 1] - v[2 * b + 1];
        if (!(dx * ey - dy * ex > 0.0)) return fail(c, REF_EINVAL, "cell %lld is not strictly convex/CCW", (long long)i);
        double len = sqrt(dx * dx + dy * dy);
        double nx = dy / len, ny = -dx / len;
        double *f = c->lfn + 4 * (s0 + k);
        f[0] = nx;
        f[1] = ny;
        f[2] = nx * v[2 * a] + ny * v[2 * a + 1];
        f[3] = len;
        c->cvtx[s0 + k] = a;
      }
    }
    /* match edges between cells and with the boundary list */
    edge_t *E = xcalloc((size_t)nl, sizeof(edge_t));
    for (int64_t i = 0; i < nc; ++i) {
      int64_t s0 = c->cptr[i], nv = c->cptr[i + 1] - s0;
      for (int64_t k = 0; k < nv; ++k) {
        int64_t a = m->cell_nodes[s0 + k], b = m->cell_nodes[s0 + (k + 1) % nv];
        E[s0 + k].a = a < b ? a : b;
        E[s0 + k].b = a < b ? b : a;
        E[s0 + k].cell = i;
        E[s0 + k].k = k;
      }
    }
    qsort(E, (size_t)nl, sizeof(edge_t), edge_cmp);
    edge_t *B = xcalloc((size_t)nb, sizeof(edge_t));
    for (int64_t b = 0; b < nb; ++b) {
      int64_t a = m->bface_nodes[2 * b], d = m->bface_nodes[2 * b + 1];
      B[b].a = a < d ? a : d;
      B[b].b = a < d ? d : a;
      B[b].cell = b;
      B[b].k = 0;
    }
    qsort(B, (size_t)nb, sizeof(edge_t), edge_cmp);
    int64_t ib = 0;
    for (int64_t e = 0; e < nl;) {
      if (e + 1 < nl && E[e + 1].a == E[e].a && E[e + 1].b == E[e].b) {
        if (e + 2 < nl && E[e + 2].a == E[e].a && E[e + 2].b == E[e].b) {
          free(E); free(B);
          return fail(c, REF_EINVAL, "edge shared by more than two cells");
        }
        c->lnb[c->cptr[E[e].cell] + E[e].k] = E[e + 1].cell;
        c->lnb[c->cptr[E[e + 1].cell] + E[e + 1].k] = E[e].cell;
        e += 2;
      } else {
        while (ib < nb && (B[ib].a < E[e].a || (B[ib].a == E[e].a && B[ib].b < E[e].b))) ++ib;
        if (ib >= nb || B[ib].a != E[e].a || B[ib].b != E[e].b) {
          free(E); free(B);
          return fail(c, REF_EINVAL, "open edge (%lld,%lld) not in the boundary list", (long long)E[e].a, (long long)E[e].b);
        }
        int64_t b = B[ib].cell;
        c->lnb[c->cptr[E[e].cell] + E[e].k] = -(b + 1);
        c->bcell[b] = E[e].cell;
        c->bk[b] = E[e].k;
        ++e;
      }
    }
    free(E);
    free(B);
  }
  for (int64_t b = 0; b < nb; ++b)
    if (c->bcell[b] < 0) return fail(c, REF_EINVAL, "boundary face %lld matches no cell edge", (long long)b);
  /* global faces: in order of first appearance over (cell, local face) */
  c->fL = xcalloc((size_t)nl, sizeof(int64_t));
  c->fR = xcalloc((size_t)nl, sizeof(int64_t));
  c->fkL = xcalloc((size_t)nl, sizeof(int64_t));
  c->fkR = xcalloc((size_t)nl, sizeof(int64_t));
  c->fn = xcalloc((size_t)nl * 2, sizeof(double));
  c->fs = xcalloc((size_t)nl, sizeof(double));
  c->fmid = xcalloc((size_t)nl * 2, sizeof(double));
  for (int64_t l = 0; l < nl; ++l) c->lface[l] = -1;
  int64_t nf = 0;
  for (int64_t i = 0; i < nc; ++i) {
    for (int64_t l = c->cptr[i]; l < c->cptr[i + 1]; ++l) {
      if (c->lface[l] >= 0) continue;
      int64_t f = nf++;
      int64_t k = l - c->cptr[i];
      c->lface[l] = f;
      c->fL[f] = i;
      c->fkL[f] = k;
      c->fn[2 * f] = c->lfn[4 * l];
      c->fn[2 * f + 1] = c->lfn[4 * l + 1];
      c->fs[f] = c->lfn[4 * l + 3];
      if (c->dim == 1) {
        c->fmid[2 * f] = c->nodes[k == 0 ? i : i + 1];
        c->fmid[2 * f + 1] = 0.0;
      } else {
        int64_t nv = c->cptr[i + 1] - c->cptr[i];
        int64_t a = c->cvtx[l], b = c->cvtx[c->cptr[i] + (k + 1) % nv];
        c->fmid[2 * f] = 0.5 * (c->nodes[2 * a] + c->nodes[2 * b]);
        c->fmid[2 * f + 1] = 0.5 * (c->nodes[2 * a + 1] + c->nodes[2 * b + 1]);
      }
      int64_t nb_ = c->lnb[l];
      if (nb_ >= 0) {
        c->fR[f] = nb_;
        int64_t found = -1;
        for (int64_t l2 = c->cptr[nb_]; l2 < c->cptr[nb_ + 1]; ++l2)
          if (c->lnb[l2] == i && c->lface[l2] < 0) { found = l2; break; }
        if (found < 0) return fail(c, REF_EINVAL, "inconsistent neighbour table");
        c->lface[found] = f;
        c->fkR[f] = found - c->cptr[nb_];
      } else {
        c->fR[f] = nb_;
        c->fkR[f] = -1;
      }
    }
  }
  c->nf = nf;
  return REF_OK;
}

/* cell across the face opposite to local face k (quads: k+2, 1D: 1-k), or -1 */
static int64_t opposite_cell(const ref_ctx *c, int64_t cell, int64_t k) {
  int64_t nv = c->cptr[cell + 1] - c->cptr[cell];
  int64_t ko;
  if (c->dim == 1) ko = 1 - k;
  else if (nv == 4) ko = (k + 2) % 4;
  else return -1;
  int64_t nb = c->lnb[c->cptr[cell] + ko];
  return nb >= 0 ? nb : -1;
}

/* ======================================================================== */
/* Init                                                                      */
/* ======================================================================== */

int ref_init(const ref_mesh *m, const ref_params *par, const double *W0, ref_ctx **out) {
  *out = NULL;
  if (!m || !par || !W0 || (m->dim != 1 && m->dim != 2) || m->n_cells <= 0) return REF_EINVAL;
  ref_ctx *c = xcalloc(1, sizeof(ref_ctx));
  if (!c) return REF_ENOMEM;
  c->dim = m->dim;
  c->nw = m->dim + 2;
  c->p = *par;
  c->K = 1 + par->D;
  c->N = 3 + par->D;
  if (!(par->R > 0 && par->mu_ref > 0 && par->T_ref > 0 && par->Pr > 0 && par->cfl > 0 && par->n_ref > 0 &&
        par->D >= 0 && par->D <= 64 && (par->dt_source == 0 || (par->dt_source == 1 && par->T_inf > 0)))) {
    *out = c;
    return fail(c, REF_EINVAL, "invalid parameters");
  }
  int rc = build_mesh(c, m);
  if (rc) { *out = c; return rc; }
  int64_t nc = c->nc, nw = c->nw;
  c->W = xcalloc((size_t)(nc * nw), sizeof(double));
  memcpy(c->W, W0, sizeof(double) * (size_t)(nc * nw));
  c->dt = xcalloc((size_t)nc, sizeof(double));
  c->ratio = xcalloc((size_t)c->cptr[nc], sizeof(double));
  c->rho_prev = xcalloc((size_t)nc, sizeof(double));
  c->rho_sum = xcalloc((size_t)nc, sizeof(double));
  c->rho_mean_prev = xcalloc((size_t)nc, sizeof(double));
  c->Sm = xcalloc((size_t)(nc * nw), sizeof(double));
  c->Sp = xcalloc((size_t)(nc * nw), sizeof(double));
  c->Fs = xcalloc((size_t)(c->nf * nw), sizeof(double));
  c->count = xcalloc((size_t)nc, sizeof(int32_t));
  c->wimp = xcalloc((size_t)c->nb * 3, sizeof(double));
  c->xwimp = xs_array(c->nb * 3);
  for (int64_t b = 0; b < c->nb; ++b) if (is_wall(c->btype[b])) c->nwall++;
  c->wall_b = xcalloc((size_t)c->nwall, sizeof(int64_t));
  c->wsurf_last = xcalloc((size_t)c->nwall * 3, sizeof(double));
  c->wsurf_sum = xcalloc((size_t)c->nwall * 3, sizeof(double));
  c->wsurf_ema = xcalloc((size_t)c->nwall * 3, sizeof(double));
  for (int64_t b = 0, w = 0; b < c->nb; ++b) if (is_wall(c->btype[b])) c->wall_b[w++] = b;
  c->cap = 1024;
  c->P = xcalloc((size_t)c->cap, sizeof(particle));
  *out = c;

  /* Eq. (33): dt_i = N_CFL Omega_i / sum_j (|U_i| + 3 sqrt(R T_i)) s_j from the
   * initial field (or, with dt_source = 1, with U and T of the freestream in
   * every cell); Eq. (34): dt_G = min_i dt_i (used everywhere under GTS). */
  double dtg = INFINITY;
  for (int64_t i = 0; i < nc; ++i) {
    prim_t s = prim(c, c->W + i * nw);
    if (!prim_ok(s)) return fail(c, REF_ENUMERIC, "invalid initial state in cell %lld", (long long)i);
    if (c->p.dt_source) {
      s.ux = c->p.u_inf_x;
      s.uy = c->dim == 2 ? c->p.u_inf_y : 0.0;
      s.T = c->p.T_inf;
    }
    double speed = c->dim == 2 ? sqrt(s.ux * s.ux + s.uy * s.uy) : fabs(s.ux);
    double a = speed + 3.0 * sqrt(c->p.R * s.T);
    double S = 0.0;
    for (int64_t l = c->cptr[i]; l < c->cptr[i + 1]; ++l) S += c->lfn[4 * l + 3];
    c->dt[i] = (c->p.cfl * c->vol[i]) / (a * S);
    if (c->dt[i] < dtg) dtg = c->dt[i];
  }
  if (!c->p.lts)
    for (int64_t i = 0; i < nc; ++i) c->dt[i] = dtg;
  /* directed crossing ratios dt_R / dt_L, Eq. (41) */
  for (int64_t i = 0; i < nc; ++i)
    for (int64_t l = c->cptr[i]; l < c->cptr[i + 1]; ++l)
      c->ratio[l] = c->lnb[l] >= 0 ? c->dt[c->lnb[l]] / c->dt[i] : 1.0;
  for (int64_t i = 0; i < nc; ++i) c->rho_prev[i] = c->W[i * nw];
  return REF_OK;
}

void ref_free(ref_ctx *c) {
  if (!c) return;
  void *ptrs[] = {c->nodes, c->cptr, c->cvtx, c->vol, c->cen, c->lfn, c->lnb, c->lface, c->fL, c->fR,
                  c->fkL, c->fkR, c->fn, c->fs, c->fmid, c->bcell, c->bk, c->btype, c->bdata, c->W,
                  c->dt, c->ratio, c->rho_prev, c->rho_sum, c->rho_mean_prev, c->P, c->Sm, c->Sp,
                  c->Fs, c->count, c->wall_b, c->wimp, c->wsurf_last, c->wsurf_sum, c->wsurf_ema};
  for (size_t k = 0; k < sizeof ptrs / sizeof ptrs[0]; ++k) free(ptrs[k]);
  if (c->xwimp) xs_array_free(c->xwimp, c->nb * 3);
  free(c);
}

const char *ref_last_error(const ref_ctx *c) { return c ? c->err : "no context"; }

/* ======================================================================== */
/* Particles                                                                 */
/* ======================================================================== */

static int push_particle(ref_ctx *c, const particle *q) {
  if (c->np == c->cap) {
    int64_t ncap = c->cap * 2;
    particle *P = realloc(c->P, sizeof(particle) * (size_t)ncap);
    if (!P) return fail(c, REF_ENOMEM, "particle store");
    c->P = P;
    c->cap = ncap;
  }
  c->P[c->np++] = *q;
  return REF_OK;
}

static void psi_particle(const ref_ctx *c, const particle *q, double *out) {
  double e = 0.5 * (q->u[0] * q->u[0] + q->u[1] * q->u[1] + q->u[2] * q->u[2]) + q->ei;
  out[0] = q->m;
  out[1] = q->m * q->u[0];
  if (c->dim == 2) {
    out[2] = q->m * q->u[1];
    out[3] = q->m * e;
  } else {
    out[2] = q->m * e;
  }
}

/* Position uniform in the cell (Sec. III.B).  1D: x_L + eps h.  2D: pick a fan
 * triangle (v0, v_{t+1}, v_{t+2}) with probability area/Omega, then uniform
 * barycentric coordinates, reflected when eps1 + eps2 > 1. */
static void sample_position(const ref_ctx *c, int64_t cell, uint64_t pid, int64_t step, double x[2]) {
  double e0, e1, e2, e3;
  draw2(c->p.seed, pid, step, P_POS, 0, &e0, &e1);
  if (c->dim == 1) {
    double xl = c->nodes[cell], xr = c->nodes[cell + 1];
    x[0] = xl + e0 * (xr - xl);
    x[1] = 0.0;
    return;
  }
  draw2(c->p.seed, pid, step, P_POS, 1, &e2, &e3);
  int64_t s0 = c->cptr[cell], nv = c->cptr[cell + 1] - s0;
  const double *v = c->nodes;
  int64_t i0 = c->cvtx[s0];
  double x0 = v[2 * i0], y0 = v[2 * i0 + 1];
  double target = e0 * c->vol[cell], acc = 0.0;
  int64_t t = 0;
  for (t = 0; t + 2 < nv; ++t) {
    double xa = v[2 * c->cvtx[s0 + t + 1]], ya = v[2 * c->cvtx[s0 + t + 1] + 1];
    double xb = v[2 * c->cvtx[s0 + t + 2]], yb = v[2 * c->cvtx[s0 + t + 2] + 1];
    acc += 0.5 * ((xa - x0) * (yb - y0) - (xb - x0) * (ya - y0));
    if (target < acc) break;
  }
  if (t + 2 >= nv) t = nv - 3;
  double xa = v[2 * c->cvtx[s0 + t + 1]], ya = v[2 * c->cvtx[s0 + t + 1] + 1];
  double xb = v[2 * c->cvtx[s0 + t + 2]], yb = v[2 * c->cvtx[s0 + t + 2] + 1];
  double b1 = e1, b2 = e2;
  if (b1 + b2 > 1.0) {
    b1 = 1.0 - b1;
    b2 = 1.0 - b2;
  }
  x[0] = (x0 + b1 * (xa - x0)) + b2 * (xb - x0);
  x[1] = (y0 + b1 * (ya - y0)) + b2 * (yb - y0);
}

/* Internal energy in units of R T of the D internal degrees of freedom of
 * Eq. (1): eta = |z|^2 / 2 for D standard normal deviates, taken in order
 * from Box-Muller pairs of INTERNAL draws call0, call0 + 1, ... (the second
 * deviate of the last pair unused when D is odd); |xi|^2 / 2 = R T eta. */
static double internal_eta(const ref_ctx *c, uint64_t pid, int64_t step, uint32_t call0) {
  double s = 0.0;
  for (int j = 0; 2 * j < c->p.D; ++j) {
    double e0, e1, z0, z1;
    draw2(c->p.seed, pid, step, P_INTERNAL, call0 + (uint32_t)j, &e0, &e1);
    box_muller(e0, e1, &z0, &z1);
    s += z0 * z0;
    if (2 * j + 1 < c->p.D) s += z1 * z1;
  }
  return 0.5 * s;
}

/* Three Gaussian velocity components from two VEL draws (call offset 2a). */
static void gauss3(const ref_ctx *c, uint64_t pid, int64_t step, uint32_t purpose, uint32_t call0, double z[3]) {
  double e0, e1, e2, e3, z3;
  draw2(c->p.seed, pid, step, purpose, call0, &e0, &e1);
  draw2(c->p.seed, pid, step, purpose, call0 + 1, &e2, &e3);
  box_muller(e0, e1, &z[0], &z[1]);
  box_muller(e2, e3, &z[2], &z3);
}

/* Deviation z = (u - U^h)/sqrt(R T^h) of one new collisionless particle.
 * Maxwellian of the hydrodynamic wave state (rho^h, U^h, T^h) of the cell.
 * With Pr != 1 the Shakhov target g^S of Eq. (4) is reached by
 * acceptance-rejection against that Maxwellian: the correction factor uses the
 * cell's total U, T, p and the heat flux Q of Eq. (5) tallied from the
 * retained particles; deviations beyond 6 sqrt(R T^h) are rejected. */
static void sample_deviation(ref_ctx *c, uint64_t pid, int64_t step, const double Uh[2], double Th,
                             const double *shak /* NULL or {Ux, Uy, T, p, Qx, Qy} */, double z[3]) {
  if (!shak) {
    gauss3(c, pid, step, P_VEL, 0, z);
    return;
  }
  double sig = sqrt(c->p.R * Th);
  double RT = c->p.R * shak[2];
  double cmax = 6.0 * sig;
  double du = sqrt((Uh[0] - shak[0]) * (Uh[0] - shak[0]) + (Uh[1] - shak[1]) * (Uh[1] - shak[1]));
  double cb = cmax + du;
  double qn = sqrt(shak[4] * shak[4] + shak[5] * shak[5]);
  double w = cb * cb / RT - 5.0;
  double Bnd = 1.0 + (fabs(1.0 - c->p.Pr) * qn * cb * (w > 5.0 ? w : 5.0)) / (5.0 * shak[3] * RT);
  /* Reading: at most 64 attempts.  If none is accepted, the particle takes
   * the first attempt's draw that lies within c_max (so every sample is
   * inside the truncated support of the target), or z = 0 if none does. */
  int first_in = -1;
  double zin[3] = {0.0, 0.0, 0.0};
  for (uint32_t att = 0; att < 64; ++att) {
    gauss3(c, pid, step, P_VEL, 2 * att, z);
    double dz = sqrt(z[0] * z[0] + z[1] * z[1] + z[2] * z[2]) * sig;
    double ea, eb;
    draw2(c->p.seed, pid, step, P_SHAKHOV, att, &ea, &eb);
    if (dz > cmax) continue;
    if (first_in < 0) {
      first_in = (int)att;
      for (int d = 0; d < 3; ++d) zin[d] = z[d];
    }
    double cx = (Uh[0] + sig * z[0]) - shak[0], cy = (Uh[1] + sig * z[1]) - shak[1], cz = sig * z[2];
    double c2 = cx * cx + cy * cy + cz * cz;
    double cq = c->dim == 2 ? cx * shak[4] + cy * shak[5] : cx * shak[4];
    double phi = ((1.0 - c->p.Pr) * cq) / (5.0 * shak[3] * RT) * (c2 / RT - 5.0);
    if (ea * Bnd <= 1.0 + phi) return;
  }
  c->n_capped++;
  for (int d = 0; d < 3; ++d) z[d] = zin[d];
}

/* sample_deviation for test access; returns 1 if the 64-attempt fallback
 * was taken */
int ref_sample_deviation(ref_ctx *c, uint64_t pid, int64_t step, const double Uh[2], double Th, const double *shak,
                         double z[3]) {
  int64_t before = c->n_capped;
  sample_deviation(c, pid, step, Uh, Th, shak, z);
  int capped = c->n_capped != before;
  c->n_capped = before;
  return capped;
}

/* Tracking of one particle, Eq. (28) with crossing detection.
 * Exit face = smallest t_e = (c_e - n_e . x)/(u . n_e) over faces with
 * u . n_e > 0 (t_e clamped at 0, ties to the lowest local index); a crossing
 * happens when t_e < t.  At an L -> R crossing m <- m dt_R/dt_L, Eq. (41), and
 * the remaining time t <- (t - t_e) dt_R/dt_L, Eq. (52).  Far-field/outflow:
 * the particle leaves.  Symmetry: specular.  Diffuse wall: re-emitted from the
 * wall Maxwellian at T_w with flux weighting (normal speed sqrt(-2 R T_w ln e)),
 * draws WALL (2h, 2h+1) for the h-th hit.  Returns 1 if it left the domain,
 * REF_ENUMERIC on a runaway, 0 otherwise. */
static int track(ref_ctx *c, particle *q, int64_t step, int32_t *ncross_out) {
  int64_t cell = q->cell;
  double t = q->t;
  int32_t nx = 0, hits = 0;
  for (;;) {
    int64_t s0 = c->cptr[cell], nv = c->cptr[cell + 1] - s0;
    double best = INFINITY;
    int64_t kb = -1;
    for (int64_t k = 0; k < nv; ++k) {
      const double *f = c->lfn + 4 * (s0 + k);
      double un = c->dim == 2 ? q->u[0] * f[0] + q->u[1] * f[1] : q->u[0] * f[0];
      if (!(un > 0.0)) continue;
      double xn = c->dim == 2 ? f[0] * q->x[0] + f[1] * q->x[1] : f[0] * q->x[0];
      double te = (f[2] - xn) / un;
      if (te < 0.0) te = 0.0;
      if (te < best) {
        best = te;
        kb = k;
      }
    }
    if (kb < 0 || !(best < t)) {
      q->x[0] = q->x[0] + q->u[0] * t;
      if (c->dim == 2) q->x[1] = q->x[1] + q->u[1] * t;
      q->cell = (int32_t)cell;
      q->t = 0.0;
      if (ncross_out) *ncross_out = nx;
      return 0;
    }
    if (++nx > MAX_CROSS) return REF_ENUMERIC;
    q->x[0] = q->x[0] + q->u[0] * best;
    if (c->dim == 2) q->x[1] = q->x[1] + q->u[1] * best;
    int64_t l = s0 + kb;
    int64_t nb = c->lnb[l];
    if (nb >= 0) {
      double r = c->ratio[l];
      t = (t - best) * r;
      q->m = q->m * r;
      cell = nb;
      continue;
    }
    int64_t b = -nb - 1;
    int32_t ty = c->btype[b];
    const double *f = c->lfn + 4 * l;
    t = t - best;
    if (ty == REF_BC_FARFIELD || ty == REF_BC_OUTFLOW) {
      q->cell = (int32_t)cell;
      q->flags |= F_EXIT;
      if (ncross_out) *ncross_out = nx;
      return 1;
    }
    if (ty == REF_BC_SYMMETRY) {
      if (c->dim == 2) {
        double un = q->u[0] * f[0] + q->u[1] * f[1];
        q->u[0] = q->u[0] - 2.0 * un * f[0];
        q->u[1] = q->u[1] - 2.0 * un * f[1];
      } else {
        q->u[0] = -q->u[0];
      }
      continue;
    }
    /* walls */
    double Tw = c->bdata[8 * b];
    double sw = sqrt(c->p.R * Tw);
    double e0, e1, e2, e3, z0, z1;
    draw2(c->p.seed, q->pid, step, P_WALL, (uint32_t)(2 * hits), &e0, &e1);
    draw2(c->p.seed, q->pid, step, P_WALL, (uint32_t)(2 * hits + 1), &e2, &e3);
    ++hits;
    if (ty == REF_BC_WALL_MAXWELL && !(e3 < c->bdata[8 * b + 1])) {
      /* specular part of the Maxwell wall: the impulse goes to the wall */
      double ub[3] = {q->u[0], q->u[1], q->u[2]};
      if (c->dim == 2) {
        double un = q->u[0] * f[0] + q->u[1] * f[1];
        q->u[0] = q->u[0] - 2.0 * un * f[0];
        q->u[1] = q->u[1] - 2.0 * un * f[1];
      } else {
        q->u[0] = -q->u[0];
      }
      xs_add(&c->xwimp[3 * b + 0], q->m * (ub[0] - q->u[0]));
      xs_add(&c->xwimp[3 * b + 1], q->m * (ub[1] - q->u[1]));
      continue;
    }
    /* diffuse re-emission; internal energy from the wall temperature */
    double vn = sqrt(-2.0 * c->p.R * Tw * log(e0));
    box_muller(e1, e2, &z0, &z1);
    double ub[3] = {q->u[0], q->u[1], q->u[2]};
    double eib = q->ei;
    if (c->p.D > 0)
      q->ei = (c->p.R * Tw) *
              internal_eta(c, q->pid, step, WALL_INTERNAL_CALL0 + (uint32_t)((hits - 1) * ((c->p.D + 1) / 2)));
    if (c->dim == 2) {
      double vt = sw * z0;
      q->u[0] = -vn * f[0] - vt * f[1];
      q->u[1] = -vn * f[1] + vt * f[0];
      q->u[2] = sw * z1;
    } else {
      q->u[0] = -vn * f[0];
      q->u[1] = sw * z0;
      q->u[2] = sw * z1;
    }
    double eb = 0.5 * (ub[0] * ub[0] + ub[1] * ub[1] + ub[2] * ub[2]);
    double ea = 0.5 * (q->u[0] * q->u[0] + q->u[1] * q->u[1] + q->u[2] * q->u[2]);
    xs_add(&c->xwimp[3 * b + 0], q->m * (ub[0] - q->u[0]));
    xs_add(&c->xwimp[3 * b + 1], q->m * (ub[1] - q->u[1]));
    xs_add(&c->xwimp[3 * b + 2], q->m * ((eb + eib) - (ea + q->ei)));
  }
}

int ref_track_one(ref_ctx *c, uint64_t pid, int64_t step, int32_t cell, double x[2], double u[3],
                  double *m, double t, int32_t *cell_out, int32_t *n_cross) {
  particle q;
  memset(&q, 0, sizeof q);
  q.pid = pid;
  q.cell = cell;
  q.x[0] = x[0];
  q.x[1] = x[1];
  q.u[0] = u[0];
  q.u[1] = u[1];
  q.u[2] = u[2];
  q.m = *m;
  q.t = t;
  int rc = track(c, &q, step, n_cross);
  x[0] = q.x[0];
  x[1] = q.x[1];
  u[0] = q.u[0];
  u[1] = q.u[1];
  u[2] = q.u[2];
  *m = q.m;
  *cell_out = q.cell;
  return rc;
}

static int cmp_cell_pid(const void *a, const void *b) {
  const particle *p = a, *q = b;
  if (p->cell != q->cell) return p->cell < q->cell ? -1 : 1;
  return p->pid < q->pid ? -1 : (p->pid > q->pid);
}

/* ======================================================================== */
/* One UGKWP-LTS step (Sec. III.C with the LTS changes of Sec. IV.B)         */
/* ======================================================================== */

typedef struct {
  double W[4], Wh[4]; /* face-frame-independent stored comps (dim + 2 used) */
  int hvalid;
  double tau, E, dt;
} cellstate;

/* van Leer limiter on one-sided differences; 0 unless both have one sign. */
static double van_leer(double a, double b) {
  double p = a * b;
  return p > 0.0 ? (2.0 * p) / (a + b) : 0.0;
}

static int fstate_ok(const double W[4], int K) {
  if (!(W[0] > 0.0) || !isfinite(W[0])) return 0;
  double U = W[1] / W[0], V = W[2] / W[0];
  double e = W[3] - 0.5 * W[0] * (U * U + V * V);
  (void)K;
  return e > 0.0 && isfinite(e);
}

/* Face value of side `self` (reading: MUSCL along the face normal line with
 * the van Leer limiter, one-sided differences weighted by the normal distance
 * between centroids; first order when the far neighbour is missing or the
 * limited value is not a valid Maxwellian).  xi_* are centroid coordinates
 * along n measured from the face midpoint. */
static void reconstruct(const double *Wfar, double xfar, const double *Wself, double xself,
                        const double *Wother, double xother, int K, double out[4], double slope[4]) {
  for (int q = 0; q < 4; ++q) {
    out[q] = Wself[q];
    slope[q] = 0.0;
  }
  if (!Wfar) return;
  double v[4], s[4];
  for (int q = 0; q < 4; ++q) {
    double d1 = (Wself[q] - Wfar[q]) / (xself - xfar);
    double d2 = (Wother[q] - Wself[q]) / (xother - xself);
    s[q] = van_leer(d1, d2);
    v[q] = Wself[q] - s[q] * xself;
  }
  if (!fstate_ok(v, K)) return;
  for (int q = 0; q < 4; ++q) {
    out[q] = v[q];
    slope[q] = s[q];
  }
}

/* Reading (the paper does not discuss positivity): an updated state Wn that
 * is not a valid Maxwellian (a cell emptied into vacuum) is replaced by the
 * content Sp / Omega of the particles that ended in the cell, Eq. (30), if
 * that is a valid state, else by a vacuum floor state (rho = 1e-12 rho_inf
 * at rest, T_inf).  Returns 1 if Wn was replaced. */
int ref_vacuum_guard(const ref_ctx *c, const double *Sp, double vol, double *Wn) {
  const int nw = c->nw;
  if (prim_ok(prim(c, Wn))) return 0;
  int ok = 0;
  if (Sp[0] > 0.0) {
    for (int q = 0; q < nw; ++q) Wn[q] = Sp[q] / vol;
    ok = prim_ok(prim(c, Wn));
  }
  if (!ok) {
    double rf = 1e-12 * c->p.rho_inf;
    for (int q = 0; q < nw; ++q) Wn[q] = 0.0;
    Wn[0] = rf;
    Wn[nw - 1] = 0.5 * (double)c->N * rf * c->p.R * c->p.T_inf;
  }
  return 1;
}

/* Face values and slopes of one interior face fi (normal n from L to R) for
 * the stored states of L, R and the cells LL, RR across their opposite faces
 * (NULL if none): each side reconstructed by reconstruct(), and the
 * equilibrium slope read as one central difference of the cell averages
 * along n, dW0 = (W_R - W_L)/(xi_R - xi_L).  All in the face frame. */
static void face_values(const ref_ctx *c, int64_t fi, const double *WLc, const double *WRc, const double *WLLc,
                        const double *WRRc, double WLf[4], double WRf[4], double sl[4], double sr[4],
                        double dW0[4]) {
  const double n2[2] = {c->fn[2 * fi], c->fn[2 * fi + 1]};
  int64_t L = c->fL[fi], R = c->fR[fi];
  int64_t LL = opposite_cell(c, L, c->fkL[fi]);
  int64_t RR = opposite_cell(c, R, c->fkR[fi]);
  double xL = (c->cen[2 * L] - c->fmid[2 * fi]) * n2[0] + (c->cen[2 * L + 1] - c->fmid[2 * fi + 1]) * n2[1];
  double xR = (c->cen[2 * R] - c->fmid[2 * fi]) * n2[0] + (c->cen[2 * R + 1] - c->fmid[2 * fi + 1]) * n2[1];
  double wL[4], wR[4], wLL[4], wRR[4], xLL = 0, xRR = 0;
  to_frame(c, WLc, n2, wL);
  to_frame(c, WRc, n2, wR);
  if (LL >= 0 && WLLc) {
    to_frame(c, WLLc, n2, wLL);
    xLL = (c->cen[2 * LL] - c->fmid[2 * fi]) * n2[0] + (c->cen[2 * LL + 1] - c->fmid[2 * fi + 1]) * n2[1];
  }
  if (RR >= 0 && WRRc) {
    to_frame(c, WRRc, n2, wRR);
    xRR = (c->cen[2 * RR] - c->fmid[2 * fi]) * n2[0] + (c->cen[2 * RR + 1] - c->fmid[2 * fi + 1]) * n2[1];
  }
  reconstruct(LL >= 0 && WLLc ? wLL : NULL, xLL, wL, xL, wR, xR, c->K, WLf, sl);
  reconstruct(RR >= 0 && WRRc ? wRR : NULL, xRR, wR, xR, wL, xL, c->K, WRf, sr);
  for (int q = 0; q < 4; ++q) dW0[q] = (wR[q] - wL[q]) / (xR - xL);
}

/* face_values of interior face fi from the current fields W (test access) */
int ref_face_values(const ref_ctx *c, int64_t fi, double WLf[4], double WRf[4], double sl[4], double sr[4],
                    double dW0[4]) {
  if (fi < 0 || fi >= c->nf || c->fR[fi] < 0) return REF_EINVAL;
  const int nw = c->nw;
  int64_t L = c->fL[fi], R = c->fR[fi];
  int64_t LL = opposite_cell(c, L, c->fkL[fi]);
  int64_t RR = opposite_cell(c, R, c->fkR[fi]);
  face_values(c, fi, c->W + L * nw, c->W + R * nw, LL >= 0 ? c->W + LL * nw : NULL, RR >= 0 ? c->W + RR * nw : NULL,
              WLf, WRf, sl, sr, dW0);
  return REF_OK;
}

/* geometry of face fi: out = {L, R (-(b+1) on the boundary), LL, RR (-1 if
 * none), midpoint x, y, unit normal x, y (from L to R)} */
int ref_face_geom(const ref_ctx *c, int64_t fi, double out[8]) {
  if (fi < 0 || fi >= c->nf) return REF_EINVAL;
  int64_t L = c->fL[fi], R = c->fR[fi];
  out[0] = (double)L;
  out[1] = (double)R;
  out[2] = (double)opposite_cell(c, L, c->fkL[fi]);
  out[3] = R >= 0 ? (double)opposite_cell(c, R, c->fkR[fi]) : -1.0;
  out[4] = c->fmid[2 * fi];
  out[5] = c->fmid[2 * fi + 1];
  out[6] = c->fn[2 * fi];
  out[7] = c->fn[2 * fi + 1];
  return REF_OK;
}

void ref_reconstruct(const double *Wfar, double xfar, const double Wself[4], double xself, const double Wother[4],
                     double xother, int K, double out[4], double slope[4]) {
  reconstruct(Wfar, xfar, Wself, xself, Wother, xother, K, out, slope);
}

int ref_step(ref_ctx *c, int32_t n_steps) {
  if (!c) return REF_EINVAL;
  const int nw = c->nw, dim = c->dim, K = c->K;
  const int64_t nc = c->nc, nb = c->nb, nf = c->nf;
  cellstate *cs = xcalloc((size_t)nc, sizeof(cellstate));
  cellstate *gs = xcalloc((size_t)nb, sizeof(cellstate));
  double *Qh = xcalloc((size_t)nc * 2, sizeof(double));
  double *Sret = xcalloc((size_t)(nc * nw), sizeof(double));
  /* exact sums of the tallies W^p, W^{p,-}, W^{p,+} (times Omega) and of the
   * retained particles' heat flux */
  xsum *xret = xs_array(nc * nw), *xsm = xs_array(nc * nw), *xsp = xs_array(nc * nw), *xq = xs_array(nc * 2);
  int rc = REF_OK;
  for (int32_t it = 0; it < n_steps && rc == REF_OK; ++it) {
    const int64_t n = c->step;
    memset(c->Sm, 0, sizeof(double) * (size_t)(nc * nw));
    memset(c->Sp, 0, sizeof(double) * (size_t)(nc * nw));
    memset(Sret, 0, sizeof(double) * (size_t)(nc * nw));
    memset(Qh, 0, sizeof(double) * (size_t)nc * 2);
    memset(c->wimp, 0, sizeof(double) * (size_t)nb * 3);
    for (int64_t k = 0; k < nc * nw; ++k) {
      xs_free(&xret[k]);
      xs_free(&xsm[k]);
      xs_free(&xsp[k]);
    }
    for (int64_t k = 0; k < nc * 2; ++k) xs_free(&xq[k]);
    for (int64_t k = 0; k < nb * 3; ++k) xs_free(&c->xwimp[k]);
    c->n_new = c->n_removed = c->n_exited = c->n_guard = c->n_capped = 0;

    /* (1) cell state: tau = mu/p, x = dt/tau, E = e^{-x} (Sec. IV.B) */
    for (int64_t i = 0; i < nc; ++i) {
      prim_t s = prim(c, c->W + i * nw);
      if (!prim_ok(s)) { rc = fail(c, REF_ENUMERIC, "invalid state in cell %lld at step %lld", (long long)i, (long long)n); break; }
      for (int q = 0; q < nw; ++q) cs[i].W[q] = c->W[i * nw + q];
      cs[i].tau = relax_time(c, s.rho, s.T);
      cs[i].dt = c->dt[i];
      cs[i].E = c->p.wave_only ? 0.0 : exp(-(c->dt[i] / cs[i].tau));
    }
    if (rc) break;

    /* (2) W^p from the retained particles, Eq. (24) (with the heat flux of
     * Eq. (5) relative to the cell velocity when Pr != 1), W^h = W - W^p. */
    for (int64_t k = 0; k < c->np; ++k) {
      particle *q = &c->P[k];
      double ps[4];
      psi_particle(c, q, ps);
      for (int w = 0; w < nw; ++w) xs_add(&xret[q->cell * nw + w], ps[w]);
      if (c->p.Pr != 1.0) {
        prim_t s = prim(c, c->W + q->cell * nw);
        double cx = q->u[0] - s.ux, cy = q->u[1] - s.uy, cz = q->u[2];
        double h = 0.5 * (cx * cx + cy * cy + cz * cz) + q->ei;
        xs_add(&xq[2 * q->cell], q->m * cx * h);
        xs_add(&xq[2 * q->cell + 1], q->m * cy * h);
      }
    }
    for (int64_t k = 0; k < nc * nw; ++k) Sret[k] = xs_round(&xret[k]);
    for (int64_t k = 0; k < nc * 2; ++k) Qh[k] = xs_round(&xq[k]);
    for (int64_t i = 0; i < nc; ++i) {
      for (int w = 0; w < nw; ++w) cs[i].Wh[w] = cs[i].W[w] - Sret[i * nw + w] / c->vol[i];
      prim_t h = prim(c, cs[i].Wh);
      cs[i].hvalid = prim_ok(h);
    }

    /* (3) ghost states: far field fixed, outflow copies W_i, symmetry mirrors
     * W_i and W^h_i; both sides of a boundary face use dt_i (Sec. IV.B). */
    for (int64_t b = 0; b < nb; ++b) {
      int64_t i = c->bcell[b];
      const double *f = c->lfn + 4 * (c->cptr[i] + c->bk[b]);
      cellstate *g = &gs[b];
      g->dt = c->dt[i];
      int ty = c->btype[b];
      if (ty == REF_BC_FARFIELD) {
        const double *d = c->bdata + 8 * b;
        double W[4];
        double ke = 0.5 * d[0] * (d[1] * d[1] + (dim == 2 ? d[2] * d[2] : 0.0));
        W[0] = d[0];
        W[1] = d[0] * d[1];
        if (dim == 2) W[2] = d[0] * d[2];
        W[dim + 1] = ke + 0.5 * (double)c->N * d[0] * c->p.R * d[3];
        for (int q = 0; q < nw; ++q) g->W[q] = g->Wh[q] = W[q];
        g->hvalid = 1;
        g->tau = relax_time(c, d[0], d[3]);
      } else if (ty == REF_BC_OUTFLOW) {
        for (int q = 0; q < nw; ++q) g->W[q] = g->Wh[q] = cs[i].W[q];
        g->hvalid = 1;
        g->tau = cs[i].tau;
      } else if (ty == REF_BC_SYMMETRY || ty == REF_BC_WALL_MAXWELL) {
        /* mirror state (the specular part of a Maxwell wall) */
        for (int q = 0; q < nw; ++q) { g->W[q] = cs[i].W[q]; g->Wh[q] = cs[i].Wh[q]; }
        if (dim == 2) {
          double mn = cs[i].W[1] * f[0] + cs[i].W[2] * f[1];
          g->W[1] = cs[i].W[1] - 2.0 * mn * f[0];
          g->W[2] = cs[i].W[2] - 2.0 * mn * f[1];
          double hn = cs[i].Wh[1] * f[0] + cs[i].Wh[2] * f[1];
          g->Wh[1] = cs[i].Wh[1] - 2.0 * hn * f[0];
          g->Wh[2] = cs[i].Wh[2] - 2.0 * hn * f[1];
        } else {
          g->W[1] = -cs[i].W[1];
          g->Wh[1] = -cs[i].Wh[1];
        }
        g->hvalid = cs[i].hvalid;
        g->tau = cs[i].tau;
      } else {
        g->hvalid = 0;
        g->tau = cs[i].tau;
      }
      g->E = c->p.wave_only ? 0.0 : exp(-(g->dt / g->tau));
    }

    /* (4) pre-transport set.  Retained particles keep their order (cell, pid).
     * Eq. (51): t_f = min(-tau_i ln eps, dt_i); collided if -tau_i ln eps < dt_i. */
    int64_t n_ret = c->np;
    for (int64_t k = 0; k < n_ret; ++k) {
      particle *q = &c->P[k];
      double e0, e1;
      draw2(c->p.seed, q->pid, n, P_FREE, 0, &e0, &e1);
      double s = -cs[q->cell].tau * log(e0);
      q->flags = 0;
      if (s < c->dt[q->cell]) {
        q->flags |= F_COLLIDE;
        q->t = s;
      } else {
        q->t = c->dt[q->cell];
      }
    }
    /* Eqs. (25)-(26) with dt_i: rho^hp = rho^h e^{-dt_i/tau_i},
     * N = ceil(rho^hp/rho N_ref), m = rho^hp Omega / N; position uniform in the
     * cell, velocity from the hydrodynamic wave, t_f = dt_i (Sec. IV.B).
     * pid = (step << 44) | (cell << 20) | j. */
    for (int64_t i = 0; i < nc && rc == REF_OK; ++i) {
      if (!cs[i].hvalid) continue;
      double rho_h = cs[i].Wh[0];
      double rho_hp = rho_h * cs[i].E;
      if (!(rho_hp > 0.0)) continue;
      double ratio = rho_hp / cs[i].W[0];
      double Nd = ceil(ratio * (double)c->p.n_ref);
      if (Nd > 1048575.0) { rc = fail(c, REF_EOVERFLOW, "too many particles in cell %lld", (long long)i); break; }
      int64_t N = (int64_t)Nd;
      double mk = (rho_hp * c->vol[i]) / (double)N;
      prim_t h = prim(c, cs[i].Wh);
      double Uh[2] = {h.ux, h.uy};
      double shak[6], *sp = NULL;
      if (c->p.Pr != 1.0) {
        prim_t s = prim(c, cs[i].W);
        shak[0] = s.ux; shak[1] = s.uy; shak[2] = s.T; shak[3] = s.rho * c->p.R * s.T;
        shak[4] = Qh[2 * i] / c->vol[i];
        shak[5] = Qh[2 * i + 1] / c->vol[i];
        sp = shak;
      }
      /* The new particles represent W^hp = W^h e^{-dt_i/tau_i} (Eq. (25)):
       * reading, for N >= 2 their deviations are shifted to zero mean and
       * scaled so that the set carries exactly the momentum and the thermal
       * energy (3 R T^h / 2 per unit mass) of W^hp. */
      int64_t first = c->np;
      xsum zs[3], es;
      for (int d = 0; d < 3; ++d) xs_init(&zs[d]);
      xs_init(&es);
      for (int64_t j = 0; j < N; ++j) {
        particle q;
        memset(&q, 0, sizeof q);
        q.pid = ((uint64_t)n << 44) | ((uint64_t)i << 20) | (uint64_t)j;
        q.cell = (int32_t)i;
        q.flags = F_NEW;
        q.m = mk;
        q.t = c->dt[i];
        sample_position(c, i, q.pid, n, q.x);
        sample_deviation(c, q.pid, n, Uh, h.T, sp, q.u);
        for (int d = 0; d < 3; ++d) xs_add(&zs[d], q.u[d]);
        if (c->p.D > 0) {
          q.ei = internal_eta(c, q.pid, n, 0);
          xs_add(&es, q.ei);
        }
        if ((rc = push_particle(c, &q))) break;
        c->n_new++;
      }
      if (rc) break;
      double sig = sqrt(c->p.R * h.T);
      double zm[3] = {0.0, 0.0, 0.0}, alpha = 1.0;
      if (N >= 2) {
        /* S = sum_k |z_k - zbar|^2, each particle's squared norm rounded
         * once, the sum exact */
        xsum S;
        xs_init(&S);
        for (int d = 0; d < 3; ++d) zm[d] = xs_round(&zs[d]) / (double)N;
        for (int64_t k = first; k < c->np; ++k) {
          double a0 = c->P[k].u[0] - zm[0], a1 = c->P[k].u[1] - zm[1], a2 = c->P[k].u[2] - zm[2];
          xs_add(&S, (a0 * a0 + a1 * a1) + a2 * a2);
        }
        alpha = sqrt((3.0 * (double)N) / xs_round(&S));
        xs_free(&S);
      }
      /* the internal energies are scaled the same way to carry exactly
       * D R T^h / 2 per unit mass */
      double beta = 1.0;
      if (N >= 2 && c->p.D > 0) beta = (0.5 * (double)c->p.D * (double)N) / xs_round(&es);
      for (int d = 0; d < 3; ++d) xs_free(&zs[d]);
      xs_free(&es);
      for (int64_t k = first; k < c->np; ++k) {
        double *u = c->P[k].u;
        double w0 = (u[0] - zm[0]) * alpha, w1 = (u[1] - zm[1]) * alpha, w2 = (u[2] - zm[2]) * alpha;
        u[0] = Uh[0] + sig * w0;
        u[1] = Uh[1] + sig * w1;
        u[2] = sig * w2;
        if (c->p.D > 0) c->P[k].ei = (c->p.R * h.T) * (beta * c->P[k].ei);
      }
    }
    if (rc) break;
    /* Reading (far field / outflow): the ghost cell is the slab of depth
     * d = dt_i (U_in + 6 sqrt(R T_g)) behind the face; it is sampled like an
     * interior cell (rho^hp = rho_g e^{-dt_i/tau_g}, count relative to Omega_i),
     * each particle flies straight for dt_i, and those reaching the face enter
     * cell i there (tangential position wrapped periodically along the face)
     * with their remaining time; the rest never enter. */
    for (int64_t b = 0; b < nb && rc == REF_OK; ++b) {
      int ty = c->btype[b];
      if (ty != REF_BC_FARFIELD && ty != REF_BC_OUTFLOW) continue;
      int64_t i = c->bcell[b];
      int64_t l = c->cptr[i] + c->bk[b];
      const double *f = c->lfn + 4 * l;
      cellstate *g = &gs[b];
      prim_t s = prim(c, g->W);
      double Uin = -(dim == 2 ? s.ux * f[0] + s.uy * f[1] : s.ux * f[0]);
      double depth = c->dt[i] * (Uin + 6.0 * sqrt(c->p.R * s.T));
      if (!(depth > 0.0)) continue;
      double sface = f[3];
      double Mslab = s.rho * g->E * depth * sface;
      if (!(Mslab > 0.0)) continue;
      double Nd = ceil((Mslab / (s.rho * c->vol[i])) * (double)c->p.n_ref);
      if (Nd > 1048575.0) { rc = fail(c, REF_EOVERFLOW, "too many ghost particles at face %lld", (long long)b); break; }
      int64_t N = (int64_t)Nd;
      double mk = Mslab / (double)N;
      double Ug[2] = {s.ux, s.uy};
      double xa = 0, ya = 0, xb = 0, yb = 0;
      if (dim == 2) {
        int64_t nv = c->cptr[i + 1] - c->cptr[i];
        int64_t va = c->cvtx[l], vb = c->cvtx[c->cptr[i] + (c->bk[b] + 1) % nv];
        xa = c->nodes[2 * va]; ya = c->nodes[2 * va + 1];
        xb = c->nodes[2 * vb]; yb = c->nodes[2 * vb + 1];
      } else {
        xa = c->nodes[c->bk[b] == 0 ? i : i + 1];
      }
      for (int64_t j = 0; j < N; ++j) {
        particle q;
        memset(&q, 0, sizeof q);
        q.pid = ((uint64_t)n << 44) | ((uint64_t)(nc + b) << 20) | (uint64_t)j;
        double e0, e1;
        draw2(c->p.seed, q.pid, n, P_POS, 0, &e0, &e1);
        double z[3], sg = sqrt(c->p.R * s.T);
        sample_deviation(c, q.pid, n, Ug, s.T, NULL, z);
        q.u[0] = Ug[0] + sg * z[0];
        q.u[1] = Ug[1] + sg * z[1];
        q.u[2] = sg * z[2];
        double vin = -(dim == 2 ? q.u[0] * f[0] + q.u[1] * f[1] : q.u[0] * f[0]);
        if (!(vin > 0.0)) continue;
        double tc = (e0 * depth) / vin;
        if (!(tc < c->dt[i])) continue;
        if (dim == 2) {
          double ut = q.u[1] * f[0] - q.u[0] * f[1];
          double a = e1 * sface + ut * tc;
          a = a - sface * floor(a / sface);
          double w = a / sface;
          q.x[0] = xa + w * (xb - xa);
          q.x[1] = ya + w * (yb - ya);
        } else {
          q.x[0] = xa;
        }
        q.cell = (int32_t)i;
        q.flags = F_GHOST;
        q.m = mk;
        q.t = c->dt[i] - tc;
        if (c->p.D > 0) q.ei = (c->p.R * s.T) * internal_eta(c, q.pid, n, 0);
        if ((rc = push_particle(c, &q))) break;
        c->n_new++;
      }
    }
    if (rc) break;
    c->n_total = c->np;

    /* (5) W^{p,-}: interior particles before transport, Eq. (30). */
    for (int64_t k = 0; k < c->np; ++k) {
      particle *q = &c->P[k];
      if (q->flags & F_GHOST) continue;
      double ps[4];
      psi_particle(c, q, ps);
      for (int w = 0; w < nw; ++w) xs_add(&xsm[q->cell * nw + w], ps[w]);
    }
    for (int64_t k = 0; k < nc * nw; ++k) c->Sm[k] = xs_round(&xsm[k]);
    /* (6) free transport with crossing scaling. */
    for (int64_t k = 0; k < c->np; ++k) {
      int r = track(c, &c->P[k], n, NULL);
      if (r < 0) { rc = fail(c, REF_ENUMERIC, "particle %llu did not finish tracking", (unsigned long long)c->P[k].pid); break; }
    }
    if (rc) break;
    /* (7) W^{p,+} over all particles ending inside, collided ones included,
     * Eq. (30); then remove collided and departed particles and re-sort. */
    int64_t keep = 0;
    for (int64_t k = 0; k < c->np; ++k) {
      particle *q = &c->P[k];
      if (q->flags & F_EXIT) { c->n_exited++; continue; }
      double ps[4];
      psi_particle(c, q, ps);
      for (int w = 0; w < nw; ++w) xs_add(&xsp[q->cell * nw + w], ps[w]);
      if (q->flags & F_COLLIDE) { c->n_removed++; continue; }
      c->P[keep++] = *q;
    }
    for (int64_t k = 0; k < nc * nw; ++k) c->Sp[k] = xs_round(&xsp[k]);
    for (int64_t k = 0; k < nb * 3; ++k) c->wimp[k] = xs_round(&c->xwimp[k]);
    c->np = keep;
    qsort(c->P, (size_t)c->np, sizeof(particle), cmp_cell_pid);
    memset(c->count, 0, sizeof(int32_t) * (size_t)nc);
    for (int64_t k = 0; k < c->np; ++k) c->count[c->P[k].cell]++;

    /* (8) wave fluxes per face, time averaged, Eqs. (49)-(50), times s_j. */
    for (int64_t fi = 0; fi < nf; ++fi) {
      int64_t L = c->fL[fi], R = c->fR[fi];
      const double n2[2] = {c->fn[2 * fi], c->fn[2 * fi + 1]};
      double F[4] = {0, 0, 0, 0}, Fe[4], Ff[4];
      double xL = (c->cen[2 * L] - c->fmid[2 * fi]) * n2[0] + (c->cen[2 * L + 1] - c->fmid[2 * fi + 1]) * n2[1];
      if (R >= 0) {
        double xR = (c->cen[2 * R] - c->fmid[2 * fi]) * n2[0] + (c->cen[2 * R + 1] - c->fmid[2 * fi + 1]) * n2[1];
        int64_t LL = opposite_cell(c, L, c->fkL[fi]);
        int64_t RR = opposite_cell(c, R, c->fkR[fi]);
        double hL[4], hR[4], hLL[4], hRR[4];
        double xLL = 0, xRR = 0;
        to_frame(c, cs[L].Wh, n2, hL);
        to_frame(c, cs[R].Wh, n2, hR);
        if (LL >= 0) {
          to_frame(c, cs[LL].Wh, n2, hLL);
          xLL = (c->cen[2 * LL] - c->fmid[2 * fi]) * n2[0] + (c->cen[2 * LL + 1] - c->fmid[2 * fi + 1]) * n2[1];
        }
        if (RR >= 0) {
          to_frame(c, cs[RR].Wh, n2, hRR);
          xRR = (c->cen[2 * RR] - c->fmid[2 * fi]) * n2[0] + (c->cen[2 * RR + 1] - c->fmid[2 * fi + 1]) * n2[1];
        }
        double WLf[4], WRf[4], sl[4], sr[4], dW0[4];
        face_values(c, fi, cs[L].W, cs[R].W, LL >= 0 ? cs[LL].W : NULL, RR >= 0 ? cs[RR].W : NULL, WLf, WRf, sl, sr,
                    dW0);
        double HLf[4], HRf[4], shl[4], shr[4];
        const double *pHL = NULL, *pHR = NULL;
        if (cs[L].hvalid) {
          int okf = LL >= 0 && cs[LL].hvalid && cs[R].hvalid;
          reconstruct(okf ? hLL : NULL, xLL, hL, xL, hR, xR, K, HLf, shl);
          pHL = HLf;
        }
        if (cs[R].hvalid) {
          int okf = RR >= 0 && cs[RR].hvalid && cs[L].hvalid;
          reconstruct(okf ? hRR : NULL, xRR, hR, xR, hL, xL, K, HRf, shr);
          pHR = HRf;
        }
        ref_flux_interior(WLf, WRf, dW0, pHL, pHR, shl, shr, cs[L].dt, cs[L].tau, cs[R].dt, cs[R].tau, K,
                          c->p.Pr, c->p.wave_only, Fe, Ff);
        for (int q = 0; q < 4; ++q) F[q] = Fe[q] + Ff[q];
      } else {
        int64_t b = -R - 1;
        cellstate *g = &gs[b];
        double wL[4], hL[4];
        to_frame(c, cs[L].W, n2, wL);
        to_frame(c, cs[L].Wh, n2, hL);
        if (c->btype[b] == REF_BC_WALL) {
          ref_flux_wall(wL, cs[L].hvalid ? hL : NULL, cs[L].dt, cs[L].tau, c->bdata[8 * b], c->p.R, K, c->p.wave_only, F);
        } else if (c->btype[b] == REF_BC_WALL_MAXWELL) {
          /* Maxwell's wall: alpha times the diffuse-wall flux plus (1 - alpha)
           * times the specular (mirror-state) flux */
          double Fd[4], Fs[4], wG[4], hG[4], dW0[4], z[4] = {0, 0, 0, 0};
          double a = c->bdata[8 * b + 1];
          ref_flux_wall(wL, cs[L].hvalid ? hL : NULL, cs[L].dt, cs[L].tau, c->bdata[8 * b], c->p.R, K, c->p.wave_only, Fd);
          to_frame(c, g->W, n2, wG);
          to_frame(c, g->Wh, n2, hG);
          for (int q = 0; q < 4; ++q) dW0[q] = (wG[q] - wL[q]) / (-2.0 * xL);
          ref_flux_interior(wL, wG, dW0, cs[L].hvalid ? hL : NULL, g->hvalid ? hG : NULL, z, z, cs[L].dt,
                            cs[L].tau, g->dt, g->tau, K, c->p.Pr, c->p.wave_only, Fe, Ff);
          for (int q = 0; q < 4; ++q) Fs[q] = Fe[q] + Ff[q];
          for (int q = 0; q < 4; ++q) F[q] = a * Fd[q] + (1.0 - a) * Fs[q];
        } else {
          double wG[4], hG[4], dW0[4], z[4] = {0, 0, 0, 0};
          to_frame(c, g->W, n2, wG);
          to_frame(c, g->Wh, n2, hG);
          for (int q = 0; q < 4; ++q) dW0[q] = (wG[q] - wL[q]) / (-2.0 * xL);
          ref_flux_interior(wL, wG, dW0, cs[L].hvalid ? hL : NULL, g->hvalid ? hG : NULL, z, z, cs[L].dt,
                            cs[L].tau, g->dt, g->tau, K, c->p.Pr, c->p.wave_only, Fe, Ff);
          for (int q = 0; q < 4; ++q) F[q] = Fe[q] + Ff[q];
        }
      }
      double Fl[4];
      from_frame(c, F, n2, Fl);
      for (int q = 0; q < nw; ++q) c->Fs[fi * nw + q] = Fl[q] * c->fs[fi];
    }

    /* (9) Eq. (53): W^{n+1} = W^n - dt_i/Omega_i sum_j F_j s_j + W^{fr,p}, with
     * W^{fr,p} = W^{p,+} - W^{p,-}, Eq. (29); fixed local face order. */
    for (int64_t i = 0; i < nc; ++i) {
      double acc[4] = {0, 0, 0, 0};
      for (int64_t l = c->cptr[i]; l < c->cptr[i + 1]; ++l) {
        int64_t f = c->lface[l];
        double sg = c->fL[f] == i ? 1.0 : -1.0;
        for (int q = 0; q < nw; ++q) acc[q] += sg * c->Fs[f * nw + q];
      }
      double coef = c->dt[i] / c->vol[i];
      double Wn[4];
      for (int q = 0; q < nw; ++q) {
        double frp = c->Sp[i * nw + q] / c->vol[i] - c->Sm[i * nw + q] / c->vol[i];
        Wn[q] = (c->W[i * nw + q] - coef * acc[q]) + frp;
      }
      c->n_guard += ref_vacuum_guard(c, c->Sp + i * nw, c->vol[i], Wn);
      for (int q = 0; q < nw; ++q) c->W[i * nw + q] = Wn[q];
    }
    /* (10) residuals (reading: RMS over cell area of the density change, and of
     * the change of the running mean, relative to rho_inf) */
    xsum num, den, num_avg;
    xs_init(&num);
    xs_init(&den);
    xs_init(&num_avg);
    for (int64_t i = 0; i < nc; ++i) {
      double rho = c->W[i * nw];
      double d = rho - c->rho_prev[i];
      xs_add(&num, c->vol[i] * d * d);
      xs_add(&den, c->vol[i]);
      c->rho_sum[i] += rho;
      double mean = c->rho_sum[i] / (double)(n + 1);
      double dm = n == 0 ? 0.0 : mean - c->rho_mean_prev[i];
      xs_add(&num_avg, c->vol[i] * dm * dm);
      c->rho_mean_prev[i] = mean;
      c->rho_prev[i] = rho;
    }
    c->r_inst = sqrt(xs_round(&num) / xs_round(&den)) / c->p.rho_inf;
    c->r_avg = sqrt(xs_round(&num_avg) / xs_round(&den)) / c->p.rho_inf;
    xs_free(&num);
    xs_free(&den);
    xs_free(&num_avg);

    /* surface: wall pressure, shear and heat flux (wave + particle impulses) */
    double Uinf = sqrt(c->p.u_inf_x * c->p.u_inf_x + c->p.u_inf_y * c->p.u_inf_y);
    double ex = c->p.u_inf_x / Uinf, ey = c->p.u_inf_y / Uinf;
    double fd = 0.0;
    for (int64_t w = 0; w < c->nwall; ++w) {
      int64_t b = c->wall_b[w];
      int64_t i = c->bcell[b];
      int64_t l = c->cptr[i] + c->bk[b];
      int64_t f = c->lface[l];
      const double *fl = c->lfn + 4 * l;
      double s = fl[3];
      double Fl[4], Fr[4] = {0, 0, 0, 0};
      for (int q = 0; q < nw; ++q) Fl[q] = c->Fs[f * nw + q] / s;
      double nx = fl[0], ny = dim == 2 ? fl[1] : 0.0;
      double mx = Fl[1], my = dim == 2 ? Fl[2] : 0.0, eF = Fl[dim + 1];
      double sdt = s * c->dt[i];
      double px = mx + c->wimp[3 * b] / sdt, py = my + (dim == 2 ? c->wimp[3 * b + 1] / sdt : 0.0);
      Fr[0] = px * nx + py * ny;
      Fr[1] = py * nx - px * ny;
      Fr[2] = eF + c->wimp[3 * b + 2] / sdt;
      fd += (px * ex + py * ey) * s;
      for (int q = 0; q < 3; ++q) {
        double v = Fr[q];
        c->wsurf_last[3 * w + q] = v;
        c->wsurf_sum[3 * w + q] += v;
        c->wsurf_ema[3 * w + q] = n == 0 ? v : (2.0 / 1001.0) * v + (1.0 - 2.0 / 1001.0) * c->wsurf_ema[3 * w + q];
      }
    }
    double cd = fd / (0.5 * c->p.rho_inf * Uinf * Uinf * c->p.L_ref);
    c->cd_last = cd;
    c->cd_sum += cd;
    c->cd_ema = n == 0 ? cd : (2.0 / 1001.0) * cd + (1.0 - 2.0 / 1001.0) * c->cd_ema;
    c->step = n + 1;
  }
  free(cs);
  free(gs);
  free(Qh);
  free(Sret);
  xs_array_free(xret, nc * nw);
  xs_array_free(xsm, nc * nw);
  xs_array_free(xsp, nc * nw);
  xs_array_free(xq, nc * 2);
  return rc;
}

/* ======================================================================== */
/* Getters                                                                   */
/* ======================================================================== */

int ref_get_fields(const ref_ctx *c, double *W) {
  memcpy(W, c->W, sizeof(double) * (size_t)(c->nc * c->nw));
  return REF_OK;
}

int ref_set_fields(ref_ctx *c, const double *W) {
  memcpy(c->W, W, sizeof(double) * (size_t)(c->nc * c->nw));
  return REF_OK;
}

int ref_get_dt(const ref_ctx *c, double *dt) {
  memcpy(dt, c->dt, sizeof(double) * (size_t)c->nc);
  return REF_OK;
}

int ref_get_counts(const ref_ctx *c, int32_t *count, int64_t *n_total, int64_t *n_new, int64_t *n_removed,
                   int64_t *n_exited) {
  if (count) memcpy(count, c->count, sizeof(int32_t) * (size_t)c->nc);
  if (n_total) *n_total = c->n_total;
  if (n_new) *n_new = c->n_new;
  if (n_removed) *n_removed = c->n_removed;
  if (n_exited) *n_exited = c->n_exited;
  return REF_OK;
}

static int cmp_pid(const void *a, const void *b) {
  const particle *p = a, *q = b;
  return p->pid < q->pid ? -1 : (p->pid > q->pid);
}

int ref_get_particles(const ref_ctx *c, int64_t cap, uint64_t *pid, int32_t *cell, double *m, double *x,
                      double *u, double *ei, int64_t *n) {
  *n = c->np;
  if (cap < c->np) return REF_EOVERFLOW;
  particle *tmp = xcalloc((size_t)c->np, sizeof(particle));
  memcpy(tmp, c->P, sizeof(particle) * (size_t)c->np);
  qsort(tmp, (size_t)c->np, sizeof(particle), cmp_pid);
  for (int64_t k = 0; k < c->np; ++k) {
    if (pid) pid[k] = tmp[k].pid;
    if (cell) cell[k] = tmp[k].cell;
    if (m) m[k] = tmp[k].m;
    for (int d = 0; d < c->dim; ++d) if (x) x[k * c->dim + d] = tmp[k].x[d];
    for (int d = 0; d < 3; ++d) if (u) u[k * 3 + d] = tmp[k].u[d];
    if (ei) ei[k] = tmp[k].ei;
  }
  free(tmp);
  return REF_OK;
}

int ref_set_particles(ref_ctx *c, int64_t n, const uint64_t *pid, const int32_t *cell, const double *m,
                      const double *x, const double *u, const double *ei) {
  c->np = 0;
  for (int64_t k = 0; k < n; ++k) {
    particle q;
    memset(&q, 0, sizeof q);
    if (cell[k] < 0 || cell[k] >= c->nc) return fail(c, REF_EINVAL, "particle cell out of range");
    q.pid = pid[k];
    q.cell = cell[k];
    q.m = m[k];
    for (int d = 0; d < c->dim; ++d) q.x[d] = x[k * c->dim + d];
    for (int d = 0; d < 3; ++d) q.u[d] = u[k * 3 + d];
    q.ei = ei ? ei[k] : 0.0;
    int rc = push_particle(c, &q);
    if (rc) return rc;
  }
  qsort(c->P, (size_t)c->np, sizeof(particle), cmp_cell_pid);
  return REF_OK;
}

int ref_residual(const ref_ctx *c, double *r_inst, double *r_avg, int64_t *step) {
  if (r_inst) *r_inst = c->r_inst;
  if (r_avg) *r_avg = c->r_avg;
  if (step) *step = c->step;
  return REF_OK;
}

/* C_p, C_F, C_Q of the wall faces (Sec. V.A) and the drag coefficient C_d
 * (Sec. V.B); mode 0 last step, 1 mean over all steps, 2 EMA with 2/1001. */
int ref_surface(const ref_ctx *c, int32_t mode, double *out, int64_t cap, int64_t *n_wall, double *Cd) {
  if (n_wall) *n_wall = c->nwall;
  if (c->step == 0) return REF_EINVAL;
  double Uinf = sqrt(c->p.u_inf_x * c->p.u_inf_x + c->p.u_inf_y * c->p.u_inf_y);
  double qd = 0.5 * c->p.rho_inf * Uinf * Uinf;
  double pinf = c->p.rho_inf * c->p.R * c->p.T_inf;
  if (Cd) *Cd = mode == 0 ? c->cd_last : mode == 1 ? c->cd_sum / (double)c->step : c->cd_ema;
  if (!out) return REF_OK;
  if (cap < c->nwall) return REF_EOVERFLOW;
  for (int64_t w = 0; w < c->nwall; ++w) {
    int64_t b = c->wall_b[w];
    int64_t i = c->bcell[b];
    int64_t l = c->cptr[i] + c->bk[b];
    const double *src = mode == 0 ? c->wsurf_last : mode == 1 ? c->wsurf_sum : c->wsurf_ema;
    double scale = mode == 1 ? 1.0 / (double)c->step : 1.0;
    int64_t f = c->lface[l];
    out[6 * w + 0] = c->fmid[2 * f];
    out[6 * w + 1] = c->fmid[2 * f + 1];
    out[6 * w + 2] = c->lfn[4 * l + 3];
    out[6 * w + 3] = (src[3 * w] * scale - pinf) / qd;
    out[6 * w + 4] = src[3 * w + 1] * scale / qd;
    out[6 * w + 5] = src[3 * w + 2] * scale / (qd * Uinf);
  }
  return REF_OK;
}

int ref_get_tally(const ref_ctx *c, double *Sminus, double *Splus) {
  if (Sminus) memcpy(Sminus, c->Sm, sizeof(double) * (size_t)(c->nc * c->nw));
  if (Splus) memcpy(Splus, c->Sp, sizeof(double) * (size_t)(c->nc * c->nw));
  return REF_OK;
}

int ref_get_face_flux(const ref_ctx *c, double *Fs) {
  memcpy(Fs, c->Fs, sizeof(double) * (size_t)(c->nf * c->nw));
  return REF_OK;
}

int64_t ref_n_faces(const ref_ctx *c) { return c->nf; }
int64_t ref_n_guard(const ref_ctx *c) { return c->n_guard; }
void ref_set_step(ref_ctx *c, int64_t step) { c->step = step; }
int64_t ref_n_capped(const ref_ctx *c) { return c->n_capped; }

/* Averaging state behind the residuals and the surface means: per cell the
 * last density, the running density sum and the last running mean; per wall
 * face the last, summed and EMA values of (p, tau, q); C_d last, sum, EMA.
 * Any pointer may be NULL. */
int ref_get_history(const ref_ctx *c, double *rho_prev, double *rho_sum, double *rho_mean_prev, double *wlast,
                    double *wsum, double *wema, double cd[3]) {
  size_t nc = (size_t)c->nc, nw3 = (size_t)c->nwall * 3;
  if (rho_prev) memcpy(rho_prev, c->rho_prev, nc * sizeof(double));
  if (rho_sum) memcpy(rho_sum, c->rho_sum, nc * sizeof(double));
  if (rho_mean_prev) memcpy(rho_mean_prev, c->rho_mean_prev, nc * sizeof(double));
  if (wlast) memcpy(wlast, c->wsurf_last, nw3 * sizeof(double));
  if (wsum) memcpy(wsum, c->wsurf_sum, nw3 * sizeof(double));
  if (wema) memcpy(wema, c->wsurf_ema, nw3 * sizeof(double));
  if (cd) {
    cd[0] = c->cd_last;
    cd[1] = c->cd_sum;
    cd[2] = c->cd_ema;
  }
  return REF_OK;
}

int ref_set_history(ref_ctx *c, const double *rho_prev, const double *rho_sum, const double *rho_mean_prev,
                    const double *wlast, const double *wsum, const double *wema, const double cd[3]) {
  size_t nc = (size_t)c->nc, nw3 = (size_t)c->nwall * 3;
  if (rho_prev) memcpy(c->rho_prev, rho_prev, nc * sizeof(double));
  if (rho_sum) memcpy(c->rho_sum, rho_sum, nc * sizeof(double));
  if (rho_mean_prev) memcpy(c->rho_mean_prev, rho_mean_prev, nc * sizeof(double));
  if (wlast) memcpy(c->wsurf_last, wlast, nw3 * sizeof(double));
  if (wsum) memcpy(c->wsurf_sum, wsum, nw3 * sizeof(double));
  if (wema) memcpy(c->wsurf_ema, wema, nw3 * sizeof(double));
  if (cd) {
    c->cd_last = cd[0];
    c->cd_sum = cd[1];
    c->cd_ema = cd[2];
  }
  return REF_OK;
}
