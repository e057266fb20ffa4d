// Device-side building blocks of the UGKWP-LTS step for gfx950 (FP64).
//
// Everything here is evaluated with -ffp-contract=off so that each product
// and sum is one IEEE operation, in the order written.  The operation order of
// the quantities that decide integers (sample counts, the collide flag, exit
// faces, acceptance tests) is fixed and documented next to each function.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ugk {

constexpr double kTwoPi = 6.283185307179586;
constexpr double kPi = 3.141592653589793;

// RNG purposes: counter word 3 = purpose << 24 | call index.
enum : uint32_t { kFree = 0, kPos = 1, kVel = 2, kWall = 3, kShakhov = 4, kInternal = 5 };

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): 10 rounds of two 32x32->64 multiplies
// with the key bumped by the Weyl constants between rounds.
// ---------------------------------------------------------------------------
struct u32x4 {
  uint32_t v[4];
};

__device__ __forceinline__ u32x4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                          uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c0;
    const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c2;
    const uint32_t n0 = static_cast<uint32_t>(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = static_cast<uint32_t>(p0 >> 32) ^ c3 ^ k1;
    c1 = static_cast<uint32_t>(p1);
    c3 = static_cast<uint32_t>(p0);
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return {{c0, c1, c2, c3}};
}

// 52 bits -> (k + 1/2) 2^-52: exact, inside (0, 1).
__device__ __forceinline__ double u01(uint32_t a, uint32_t b) {
  const uint64_t k = (static_cast<uint64_t>(a) << 20) | static_cast<uint64_t>(b >> 12);
  return (static_cast<double>(k) + 0.5) * 2.220446049250313e-16;
}

// Two uniforms keyed by (seed; pid, step, purpose, call).
__device__ __forceinline__ void rng2(uint64_t seed, uint64_t pid, int64_t step, uint32_t purpose, uint32_t call,
                                     double &e0, double &e1) {
  const u32x4 o = philox10(static_cast<uint32_t>(pid), static_cast<uint32_t>(pid >> 32),
                           static_cast<uint32_t>(step), (purpose << 24) | call, static_cast<uint32_t>(seed),
                           static_cast<uint32_t>(seed >> 32));
  e0 = u01(o.v[0], o.v[1]);
  e1 = u01(o.v[2], o.v[3]);
}

// Box-Muller: r = sqrt(-2 ln e0), angle 2 pi e1.
__device__ __forceinline__ void box_muller(double e0, double e1, double &z0, double &z1) {
  const double r = sqrt(-2.0 * log(e0));
  const double a = kTwoPi * e1;
  z0 = r * cos(a);
  z1 = r * sin(a);
}

// Three standard normals from calls (c, c + 1).
__device__ __forceinline__ void gauss3(uint64_t seed, uint64_t pid, int64_t step, uint32_t purpose, uint32_t c,
                                       double z[3]) {
  double e0, e1, e2, e3, spare;
  rng2(seed, pid, step, purpose, c, e0, e1);
  rng2(seed, pid, step, purpose, c + 1, e2, e3);
  box_muller(e0, e1, z[0], z[1]);
  box_muller(e2, e3, z[2], spare);
}

// Internal energy in units of R T of D internal degrees of freedom (the
// Maxwellian's internal part, Eq. (1)): half the sum of squares of D standard
// normal deviates, taken in order from Box-Muller pairs of INTERNAL draws
// call0, call0 + 1, ... (the second deviate of the last pair unused when D is
// odd).  Birth uses calls from 0, the h-th wall hit calls from
// kWallInternalCall0 + h ceil(D/2).
constexpr uint32_t kWallInternalCall0 = 256;
__device__ __forceinline__ double internal_eta(uint64_t seed, uint64_t pid, int64_t step, uint32_t call0, int D) {
  double s = 0.0;
  for (int j = 0; 2 * j < D; ++j) {
    double e0, e1, z0, z1;
    rng2(seed, pid, step, kInternal, call0 + static_cast<uint32_t>(j), e0, e1);
    box_muller(e0, e1, z0, z1);
    s += z0 * z0;
    if (2 * j + 1 < D) s += z1 * z1;
  }
  return 0.5 * s;
}

// ---------------------------------------------------------------------------
// Normalized time-integration coefficients of one cell side, Eq. (16) / dt
// (Eq. (48)), with x = dt/tau, E = e^-x, phi = (1 - E)/x:
//   a = 1 - phi, b = tau (2 phi - 1 - E), c = tau (x/2 - 1 + phi),
//   d = phi, e = tau (E - phi); free-transport wave (Eq. (50)):
//   f0 = d - E, f1 = e + dt E / 2 = tau (E - phi + x E / 2).
// Below x = 1 each combination is summed from its series in t_k = (-x)^k/(k+1)!
// (largest index first) to avoid cancellation.
// ---------------------------------------------------------------------------
struct Coef {
  double a, b, c, d, e, E, f0, f1;
};

__device__ __forceinline__ Coef time_coef(double dt, double tau) {
  const double x = dt / tau;
  const double E = exp(-x);
  Coef r;
  r.E = E;
  if (x < 1.0) {
    constexpr int kMax = 30;
    double t[kMax + 1];
    t[0] = 1.0;
#pragma unroll
    for (int k = 1; k <= kMax; ++k) t[k] = t[k - 1] * (-x) / static_cast<double>(k + 1);
    double sphi = 0.0, sa = 0.0, sc = 0.0, sb = 0.0, se = 0.0, sg = 0.0;
#pragma unroll
    for (int k = kMax; k >= 0; --k) {
      sphi += t[k];
      if (k >= 1) {
        sa += t[k];
        se += static_cast<double>(k) * t[k];
      }
      if (k >= 2) {
        sc += t[k];
        sb += static_cast<double>(1 - k) * t[k];
        sg += 0.5 * static_cast<double>(k * (1 - k)) * t[k];
      }
    }
    r.d = sphi;
    r.a = -sa;
    r.c = tau * sc;
    r.b = tau * sb;
    r.e = tau * se;
    r.f0 = -se;
    r.f1 = tau * sg;
  } else {
    const double phi = (1.0 - E) / x;
    r.d = phi;
    r.a = 1.0 - phi;
    r.b = tau * ((2.0 * phi - 1.0) - E);
    r.c = tau * ((0.5 * x - 1.0) + phi);
    r.e = tau * (E - phi);
    r.f0 = phi - E;
    r.f1 = tau * ((E - phi) + 0.5 * x * E);
  }
  return r;
}

// ---------------------------------------------------------------------------
// Maxwellian moments in the face frame (u_n normal, u_t tangential, K lumped
// degrees of freedom xi).  lambda = 1/(2RT).
// ---------------------------------------------------------------------------
struct Mom {
  double n[7];  // <u_n^k>, k = 0..6, half range (sign +/-1) or full (0)
  double t[5];  // <u_t^k>, k = 0..4
  double x[3];  // <xi^(2k)>, k = 0..2
};

__device__ __forceinline__ void moments(Mom &m, double U, double V, double lam, int K, int sign) {
  if (sign == 0) {
    m.n[0] = 1.0;
    m.n[1] = U;
  } else {
    const double sl = sqrt(lam);
    const double ex = exp(-lam * U * U) / (2.0 * sqrt(kPi * lam));
    if (sign > 0) {
      m.n[0] = 0.5 * erfc(-sl * U);
      m.n[1] = U * m.n[0] + ex;
    } else {
      m.n[0] = 0.5 * erfc(sl * U);
      m.n[1] = U * m.n[0] - ex;
    }
  }
#pragma unroll
  for (int k = 0; k + 2 <= 6; ++k) m.n[k + 2] = U * m.n[k + 1] + static_cast<double>(k + 1) / (2.0 * lam) * m.n[k];
  m.t[0] = 1.0;
  m.t[1] = V;
#pragma unroll
  for (int k = 0; k + 2 <= 4; ++k) m.t[k + 2] = V * m.t[k + 1] + static_cast<double>(k + 1) / (2.0 * lam) * m.t[k];
  m.x[0] = 1.0;
  m.x[1] = static_cast<double>(K) / (2.0 * lam);
  m.x[2] = static_cast<double>(K * (K + 2)) / (4.0 * lam * lam);
}

__device__ __forceinline__ double mom3(const Mom &m, int a, int b, int d) { return m.n[a] * m.t[b] * m.x[d]; }

// <u_n^a u_t^b xi^2d Psi>, Psi = (1, u_n, u_t, (u_n^2 + u_t^2 + xi^2)/2).
__device__ __forceinline__ void psi_mom(const Mom &m, int a, int b, int d, double o[4]) {
  o[0] = mom3(m, a, b, d);
  o[1] = mom3(m, a + 1, b, d);
  o[2] = mom3(m, a, b + 1, d);
  o[3] = 0.5 * (mom3(m, a + 2, b, d) + mom3(m, a, b + 2, d) + mom3(m, a, b, d + 1));
}

// <u_n^a Psi (c0 + cn u_n + ct u_t + c4 (u^2 + xi^2)/2)>.
__device__ __forceinline__ void psi_poly(const Mom &m, int a, const double c[4], double o[4]) {
  double t0[4], t1[4], t2[4], t3[4], t4[4], t5[4];
  psi_mom(m, a, 0, 0, t0);
  psi_mom(m, a + 1, 0, 0, t1);
  psi_mom(m, a, 1, 0, t2);
  psi_mom(m, a + 2, 0, 0, t3);
  psi_mom(m, a, 2, 0, t4);
  psi_mom(m, a, 0, 1, t5);
#pragma unroll
  for (int q = 0; q < 4; ++q)
    o[q] = c[0] * t0[q] + c[1] * t1[q] + c[2] * t2[q] + c[3] * (0.5 * (t3[q] + t4[q] + t5[q]));
}

struct FState {
  double rho, U, V, lam;
};

// Face-frame W = (rho, rho U, rho V, rho E): lambda = (K + 2) rho / (4 e).
__device__ __forceinline__ FState fstate(const double W[4], int K) {
  FState s;
  s.rho = W[0];
  s.U = W[1] / W[0];
  s.V = W[2] / W[0];
  const double e = W[3] - 0.5 * s.rho * (s.U * s.U + s.V * s.V);
  s.lam = (static_cast<double>(K + 2) * s.rho) / (4.0 * e);
  return s;
}

__device__ __forceinline__ bool fstate_ok(const double W[4]) {
  if (!(W[0] > 0.0) || !isfinite(W[0])) return false;
  const double U = W[1] / W[0], V = W[2] / W[0];
  const double e = W[3] - 0.5 * W[0] * (U * U + V * V);
  return e > 0.0 && isfinite(e);
}

// Coefficients of d ln g / dn (Eqs. (18)-(19)) for the conservative normal
// derivative dW; lambda' divided by Pr (Prandtl correction, Sec. III.A).
__device__ __forceinline__ void microslope(const double W[4], const double dW[4], int K, double Pr, double a[4]) {
  const FState s = fstate(W, K);
  const double N = static_cast<double>(K + 2);
  const double rho = s.rho, U = s.U, V = s.V, lam = s.lam;
  const double dU = (dW[1] - U * dW[0]) / rho;
  const double dV = (dW[2] - V * dW[0]) / rho;
  const double e = W[3] - 0.5 * rho * (U * U + V * V);
  const double de = (dW[3] - 0.5 * dW[0] * (U * U + V * V)) - rho * (U * dU + V * dV);
  double dlam = N * (dW[0] * e - rho * de) / (4.0 * e * e);
  dlam = dlam / Pr;
  a[3] = -2.0 * dlam;
  a[1] = 2.0 * (dlam * U + lam * dU);
  a[2] = 2.0 * (dlam * V + lam * dV);
  a[0] = ((dW[0] / rho + 0.5 * N * (dlam / lam)) - dlam * (U * U + V * V)) - 2.0 * lam * (U * dU + V * dV);
}

// Interior-face time-averaged flux, face frame: equilibrium part Eq. (49)
// with W0 from Eq. (17), a from the continuous normal slope dW0, A from
// Eq. (22); free-transport wave part Eq. (50) read upwind (left hydrodynamic
// state for u_n > 0, right for u_n < 0); a side whose flag hasL / hasR is
// false adds none.  (Flags rather than null pointers keep the arrays in
// registers.)
__device__ __forceinline__ void flux_interior(const double (&WL)[4], const double (&WR)[4], const double (&dW0)[4],
                                              bool hasL, const double (&WhL)[4], bool hasR, const double (&WhR)[4],
                                              const double (&dWhL)[4], const double (&dWhR)[4], double dtL,
                                              double tauL, double dtR, double tauR, int K, double Pr, int wave_only,
                                              double (&F)[4]) {
  const FState sL = fstate(WL, K), sR = fstate(WR, K);
  Mom m;
  double pL[4], pR[4], W0[4];
  moments(m, sL.U, sL.V, sL.lam, K, +1);
  psi_mom(m, 0, 0, 0, pL);
  moments(m, sR.U, sR.V, sR.lam, K, -1);
  psi_mom(m, 0, 0, 0, pR);
#pragma unroll
  for (int q = 0; q < 4; ++q) W0[q] = sL.rho * pL[q] + sR.rho * pR[q];
  const FState s0 = fstate(W0, K);
  Coef cL = time_coef(dtL, tauL), cR = time_coef(dtR, tauR);
  if (wave_only) {  // no particles take a share of the free transport
    cL.f0 = cL.d;
    cL.f1 = cL.e;
    cR.f0 = cR.d;
    cR.f1 = cR.e;
  }
  double Feq[4] = {0.0, 0.0, 0.0, 0.0};
  // an interface the two sides leave so fast that it holds no gas in FP64
  // (W0's density below 1e-30 of theirs or not a valid Maxwellian) carries
  // no equilibrium flux; neither does a non-finite one
  if (W0[0] > 1e-30 * (sL.rho + sR.rho) && s0.lam > 0.0 && s0.lam < INFINITY) {
    double a[4], A[4], Wt[4], tmp[4];
    microslope(W0, dW0, K, Pr, a);
    moments(m, s0.U, s0.V, s0.lam, K, 0);
    psi_poly(m, 1, a, tmp);
#pragma unroll
    for (int q = 0; q < 4; ++q) Wt[q] = -s0.rho * tmp[q];
    microslope(W0, Wt, K, 1.0, A);
    double f1[4], fa[4], fA[4];
    moments(m, s0.U, s0.V, s0.lam, K, +1);
    psi_mom(m, 1, 0, 0, f1);
    psi_poly(m, 2, a, fa);
    psi_poly(m, 1, A, fA);
#pragma unroll
    for (int q = 0; q < 4; ++q) Feq[q] = s0.rho * ((cL.a * f1[q] + cL.b * fa[q]) + cL.c * fA[q]);
    moments(m, s0.U, s0.V, s0.lam, K, -1);
    psi_mom(m, 1, 0, 0, f1);
    psi_poly(m, 2, a, fa);
    psi_poly(m, 1, A, fA);
#pragma unroll
    for (int q = 0; q < 4; ++q) Feq[q] = Feq[q] + s0.rho * ((cR.a * f1[q] + cR.b * fa[q]) + cR.c * fA[q]);
    if (!isfinite(Feq[0]) || !isfinite(Feq[1]) || !isfinite(Feq[2]) || !isfinite(Feq[3])) {
#pragma unroll
      for (int q = 0; q < 4; ++q) Feq[q] = 0.0;
    }
  }
  double Ffr[4] = {0.0, 0.0, 0.0, 0.0};
  if (hasL) {
    const FState h = fstate(WhL, K);
    double ah[4], g1[4], ga[4];
    microslope(WhL, dWhL, K, 1.0, ah);
    moments(m, h.U, h.V, h.lam, K, +1);
    psi_mom(m, 1, 0, 0, g1);
    psi_poly(m, 2, ah, ga);
#pragma unroll
    for (int q = 0; q < 4; ++q) Ffr[q] += h.rho * (cL.f0 * g1[q] + cL.f1 * ga[q]);
  }
  if (hasR) {
    const FState h = fstate(WhR, K);
    double ah[4], g1[4], ga[4];
    microslope(WhR, dWhR, K, 1.0, ah);
    moments(m, h.U, h.V, h.lam, K, -1);
    psi_mom(m, 1, 0, 0, g1);
    psi_poly(m, 2, ah, ga);
#pragma unroll
    for (int q = 0; q < 4; ++q) Ffr[q] += h.rho * (cR.f0 * g1[q] + cR.f1 * ga[q]);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) F[q] = Feq[q] + Ffr[q];
}

// Diffuse isothermal wall, first order: outgoing half (into the wall)
// abar g(W) + (dbar - E) g(W^h); reflected half: wall Maxwellian at rest and
// T_w with the density that makes the net wave mass flux zero.
__device__ __forceinline__ void flux_wall(const double (&W)[4], bool hasWh, const double (&Wh)[4], double dt,
                                          double tau, double Tw, double R, int K, int wave_only, double (&F)[4]) {
  Coef co = time_coef(dt, tau);
  if (wave_only) {
    co.f0 = co.d;
    co.f1 = co.e;
  }
  Mom m;
  double t[4];
  const FState s = fstate(W, K);
  moments(m, s.U, s.V, s.lam, K, +1);
  psi_mom(m, 1, 0, 0, t);
#pragma unroll
  for (int q = 0; q < 4; ++q) F[q] = s.rho * co.a * t[q];
  if (hasWh) {
    const FState h = fstate(Wh, K);
    moments(m, h.U, h.V, h.lam, K, +1);
    psi_mom(m, 1, 0, 0, t);
#pragma unroll
    for (int q = 0; q < 4; ++q) F[q] += h.rho * co.f0 * t[q];
  }
  const double lw = 1.0 / (2.0 * R * Tw);
  moments(m, 0.0, 0.0, lw, K, -1);
  psi_mom(m, 1, 0, 0, t);
  const double rw = F[0] / (-t[0]);
#pragma unroll
  for (int q = 0; q < 4; ++q) F[q] += rw * t[q];
}

// van Leer limiter: 0 unless both one-sided slopes share a sign.
__device__ __forceinline__ double van_leer(double a, double b) {
  const double p = a * b;
  return p > 0.0 ? (2.0 * p) / (a + b) : 0.0;
}

// Face value along the normal line (face at xi = 0): limited slope from the
// far neighbour and the other side; first order if there is no far neighbour
// (has_far false) or the limited value is not a valid Maxwellian.
__device__ __forceinline__ void reconstruct(bool has_far, const double (&Wfar)[4], double xfar,
                                            const double (&Wself)[4], double xself, const double (&Wother)[4],
                                            double xother, double (&out)[4], double (&slope)[4]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    out[q] = Wself[q];
    slope[q] = 0.0;
  }
  if (!has_far) return;
  double v[4], s[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const double d1 = (Wself[q] - Wfar[q]) / (xself - xfar);
    const double d2 = (Wother[q] - Wself[q]) / (xother - xself);
    s[q] = van_leer(d1, d2);
    v[q] = Wself[q] - s[q] * xself;
  }
  if (!fstate_ok(v)) return;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    out[q] = v[q];
    slope[q] = s[q];
  }
}

// ---------------------------------------------------------------------------
// Wavefront (64-lane) helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ int lane_id() { return static_cast<int>(threadIdx.x & 63u); }

// ---------------------------------------------------------------------------
// Order-independent sums.  The particle tallies of Eqs. (24), (29)-(30), the
// wall impulses and the residual sums are accumulated in fixed point: a term
// v is cut into NL 32-bit chunks of a window [2^(E - 32 NL), 2^E),
//   v = sum_j c_j 2^(E - 32 NL + 32 j),  c_j integer, |c_j| < 2^32,
// each chunk held in an FP64 value (bits of v below the window are dropped).
// Sums of up to 2^20 chunks stay below 2^52 and are exact in FP64, so a
// chunk total does not depend on the order in which the terms arrive
// (lane-strided loops, wavefront trees or atomics).  The total is rounded
// once to the FP64 value nearest the window's exact sum (ties to even).
// Each accumulated quantity has its own window E, fixed at init.  The
// tallies use NL = 6: a 192-bit window keeps every particle term of any cell
// (particle masses span some 30 decades between a stagnation layer and a
// near-vacuum wake) exact to far below an ulp of its cell's content, so the
// rounded tally is that of the exact sum; the others use NL = 4.
// ---------------------------------------------------------------------------
constexpr int kMaxLimbs = 6;
struct XWin {
  double down;           // 2^(32 - E): scales a term so that its top chunk is the integer part
  double up[kMaxLimbs];  // 2^(E - 32 NL + 32 j): weight of chunk j
};

constexpr double kTwo32 = 4294967296.0;
constexpr double kTwoM32 = 1.0 / 4294967296.0;

// Chunks of v in window w; returns false if |v| >= 2^E or v is not finite.
template <int NL>
__device__ __forceinline__ bool xs_split(double v, const XWin &w, double c[NL]) {
  double t = v * w.down;
  const bool ok = fabs(t) < kTwo32;
#pragma unroll
  for (int j = NL - 1; j > 0; --j) {
    c[j] = trunc(t);
    t = (t - c[j]) * kTwo32;
  }
  c[0] = trunc(t);
  return ok;
}

// Carry-normalizes chunk totals L (|L_j| < 2^52): L_0..L_{NL-2} in
// [0, 2^32), the sign in L_{NL-1}.  Exact.
template <int NL>
__device__ __forceinline__ void xs_normalize(double L[NL]) {
#pragma unroll
  for (int j = 0; j < NL - 1; ++j) {
    const double cy = floor(L[j] * kTwoM32);
    L[j] = L[j] - cy * kTwo32;
    L[j + 1] = L[j + 1] + cy;
  }
}

// The FP64 value nearest sum_j L_j 2^(E - 32 NL + 32 j) (ties to even).
// After normalization the nonzero chunks are nonoverlapping partials of
// increasing magnitude; they are added from the top, and an exact half-way
// case is settled by the sign of the next partial below (the final step of
// Shewchuk's exactly rounded summation, 1997).
template <int NL>
__device__ __forceinline__ double xs_round(const double Lin[NL], const XWin &w) {
  double L[NL];
#pragma unroll
  for (int j = 0; j < NL; ++j) L[j] = Lin[j];
  xs_normalize<NL>(L);
  double p[NL];
  int n = 0;
#pragma unroll
  for (int j = 0; j < NL; ++j)
    if (L[j] != 0.0) p[n++] = L[j] * w.up[j];
  if (n == 0) return 0.0;
  double hi = p[--n], lo = 0.0;
  while (n > 0) {
    const double x = hi, y = p[--n];
    hi = x + y;
    const double yr = hi - x;
    lo = y - yr;
    if (lo != 0.0) break;
  }
  if (n > 0 && ((lo < 0.0 && p[n - 1] < 0.0) || (lo > 0.0 && p[n - 1] > 0.0))) {
    const double y = lo * 2.0;
    const double x = hi + y;
    const double yr = x - hi;
    if (y == yr) hi = x;
  }
  return hi;
}

// One halving exchange: lanes with bit `o` set keep v[H..2H), the others
// v[0..H), each adding its partner's copy; the kept half moves to v[0..H).
template <int H, int P>
__device__ __forceinline__ void spread_step(double (&v)[P], int o, bool hi) {
#pragma unroll
  for (int j = 0; j < H; ++j) {
    const double send = hi ? v[j] : v[j + H];
    const double keep = hi ? v[j + H] : v[j];
    v[j] = keep + __shfl_xor(send, o, 64);
  }
  if constexpr (H > 1) spread_step<H / 2>(v, o >> 1, (lane_id() & (o >> 1)) != 0);
}

template <int P>
__device__ __forceinline__ double wave_sum_spread(double (&v)[P]) {
  static_assert(P >= 2 && P <= 64 && (P & (P - 1)) == 0, "P: a power of two in [2, 64]");
  spread_step<P / 2>(v, 32, (lane_id() & 32) != 0);
  // the remaining exchanges are plain sums
#pragma unroll
  for (int o = 32 / (P / 2) / 2; o >= 1; o >>= 1) v[0] += __shfl_xor(v[0], o, 64);
  return v[0];
}

template <int P>
__host__ __device__ constexpr int spread_shift() {
  return P == 64 ? 0 : P == 32 ? 1 : P == 16 ? 2 : P == 8 ? 3 : P == 4 ? 4 : P == 2 ? 5 : 6;
}

__device__ __forceinline__ int popc_below(uint64_t mask) {
  const int l = lane_id();
  const uint64_t lt = l == 0 ? 0ull : (~0ull >> (64 - l));
  return __popcll(mask & lt);
}

}  // namespace ugk
