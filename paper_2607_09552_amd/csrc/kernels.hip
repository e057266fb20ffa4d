// HIP kernels of the UGKWP-LTS step for gfx950 (CDNA4, 64-lane wavefronts).
//
// Particle store: structure of arrays (x, y, ux, uy, uz, m: f64; pid: u64;
// cell: i32), double-buffered, sorted by cell at the start of every step.
// The pre-transport set is [retained | new from cells | entered from ghosts].
#include "kernels.h"

#include <type_traits>

namespace ugk {

// ---------------------------------------------------------------------------
// Small helpers
// ---------------------------------------------------------------------------
template <int DIM>
struct Prim {
  double rho, ux, uy, T, e;
};

// rho, U from W; e = rho E - rho |U|^2 / 2; T = 2 e / (N R rho), N = 3 + D.
template <int DIM>
__device__ __forceinline__ Prim<DIM> prim(const double *W, double NR) {
  Prim<DIM> s;
  s.rho = W[0];
  s.ux = W[1] / s.rho;
  s.uy = DIM == 2 ? W[2] / s.rho : 0.0;
  const double ke = 0.5 * s.rho * (s.ux * s.ux + s.uy * s.uy);
  s.e = W[DIM + 1] - ke;
  s.T = (2.0 * s.e) / (NR * s.rho);
  return s;
}

template <int DIM>
__device__ __forceinline__ bool prim_ok(const Prim<DIM> &s) {
  return s.rho > 0.0 && s.e > 0.0 && isfinite(s.rho) && isfinite(s.e);
}

// tau = mu / p (Eq. (3)), mu = mu_ref (T / T_ref)^omega.
__device__ __forceinline__ double relax_time(const Params &p, double mu_ref, double rho, double T) {
  const double mu = mu_ref * pow(T / p.T_ref, p.omega);
  return mu / (rho * p.R * T);
}

// Cases of a batch: every case is computed as if alone.  A particle's pid
// uses its case's local cell and boundary-face numbering and its random
// numbers its case's seed.
__device__ __forceinline__ int case_of(const Geo &g, int64_t cell) { return g.ccase ? g.ccase[cell] : 0; }
__device__ __forceinline__ uint64_t case_seed(const Geo &g, const Params &p, int cs) {
  return g.ccase ? g.case_seed[cs] : p.seed;
}
__device__ __forceinline__ double case_val(const Geo &g, int cs, int k, double single) {
  return g.ccase ? g.case_par[cs * kCaseN + k] : single;
}

template <int DIM>
__device__ __forceinline__ void to_frame(const double *W, double nx, double ny, double o[4]) {
  o[0] = W[0];
  if (DIM == 2) {
    o[1] = W[1] * nx + W[2] * ny;
    o[2] = W[2] * nx - W[1] * ny;
    o[3] = W[3];
  } else {
    o[1] = W[1] * nx;
    o[2] = 0.0;
    o[3] = W[2];
  }
}

template <int DIM>
__device__ __forceinline__ void from_frame(const double F[4], double nx, double ny, double *o) {
  o[0] = F[0];
  if (DIM == 2) {
    o[1] = F[1] * nx - F[2] * ny;
    o[2] = F[1] * ny + F[2] * nx;
    o[3] = F[3];
  } else {
    o[1] = F[1] * nx;
    o[2] = F[3];
  }
}

// Groups the lanes of a wavefront by key (destination cell >= 0; -1 = none):
// returns the lane mask of the caller's group and sets `leader` to its lowest
// lane.  Integer work only (ballot and readlane).
__device__ __forceinline__ uint64_t wave_group(int key, int &leader) {
  uint64_t todo = __ballot(key >= 0), mine = 0;
  leader = -1;
  while (todo) {
    const int l = __ffsll(static_cast<long long>(todo)) - 1;
    const int k = __builtin_amdgcn_readlane(key, l);
    const uint64_t same = __ballot(key == k);
    if (key == k) {
      mine = same;
      leader = l;
    }
    todo &= ~same;
  }
  return mine;
}

// Mixed-precision store: positions relative to the cell's anchor.
template <class R> struct IsF32 { static constexpr bool value = false; };
template <> struct IsF32<float> { static constexpr bool value = true; };

// Writes a global position (x, y) of a particle in `cell` to slot k: as is in
// the FP64 store, relative to the cell's anchor in the FP32 store.
template <int DIM, class R>
__device__ __forceinline__ void store_position(const Geo &g, const StoreT<R> &s, int64_t k, int64_t cell, double x,
                                               double y) {
  if constexpr (IsF32<R>::value) {
    const double2 a = g.anchor[cell];
    s.x[k] = static_cast<float>(x - a.x);
    if (DIM == 2) s.y[k] = static_cast<float>(y - a.y);
  } else {
    s.x[k] = x;
    if (DIM == 2) s.y[k] = y;
  }
}

// ---------------------------------------------------------------------------
// a1: local time step from the initial field, Eq. (33), and Eq. (34)
// ---------------------------------------------------------------------------
template <int DIM>
__global__ void k_init_dt(Geo g, Params p, const double *__restrict__ W, double *__restrict__ dt,
                          int *__restrict__ flags) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= g.nc) return;
  const Prim<DIM> s = prim<DIM>(W + i * (DIM + 2), p.NR);
  if (!prim_ok(s)) {
    atomicOr(flags, kFlagInvalid);
    dt[i] = 0.0;
    return;
  }
  const double speed = DIM == 2 ? sqrt(s.ux * s.ux + s.uy * s.uy) : fabs(s.ux);
  const double a = speed + 3.0 * sqrt(p.R * s.T);
  double S = 0.0;
  for (int k = 0; k < g.NV; ++k) {
    const int64_t l = i * g.NV + k;
    if (g.lnb[l] == kPad) continue;
    S += g.lfs[l];
  }
  dt[i] = (p.cfl * g.vol[i]) / (a * S);
}

// dt_i <- min_j dt_j under GTS; directed crossing ratios dt_R / dt_L (Eq. (41)).
__global__ void k_init_ratio(Geo g, const double *__restrict__ dt, double4 *__restrict__ lfn) {
  const int64_t l = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (l >= g.nc * g.NV) return;
  const int64_t i = l / g.NV;
  const int nb = g.lnb[l];
  lfn[l].w = nb >= 0 ? dt[nb] / dt[i] : 1.0;
}

// Mixed-precision tables: FP32 face data with offsets relative to the cell's
// anchor, and the shift of anchors to the neighbour across each face (the
// position of a particle crossing into it, relative to the new anchor, is
// the old relative position plus this shift).
__global__ void k_init_mixed(Geo g, float4 *__restrict__ lfn32, float2 *__restrict__ lda) {
  const int64_t l = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (l >= g.nc * g.NV) return;
  const int64_t i = l / g.NV;
  const double4 f = g.lfn[l];
  const double2 a = g.anchor[i];
  lfn32[l] = make_float4(static_cast<float>(f.x), static_cast<float>(f.y),
                         static_cast<float>(f.z - (f.x * a.x + f.y * a.y)), static_cast<float>(f.w));
  const int nb = g.lnb[l];
  float2 d = make_float2(0.0f, 0.0f);
  if (nb >= 0) {
    const double2 b = g.anchor[nb];
    d = make_float2(static_cast<float>(a.x - b.x), static_cast<float>(a.y - b.y));
  }
  lda[l] = d;
}

// ---------------------------------------------------------------------------
// a2: cell preparation.  tau_i, E_i = e^{-dt_i/tau_i}, W^h = W - W^p
// (Eq. (24)), and the count of new particles N = ceil(rho^hp / rho N_ref)
// with rho^hp = rho^h E_i and mass m = rho^hp Omega_i / N (Eqs. (25)-(26)).
// ---------------------------------------------------------------------------
template <int DIM>
__global__ void k_cell_prep(Geo g, Params p, State st) {
  constexpr int NW = DIM + 2;
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= g.nc || *st.halt) return;
  const double *W = st.W + i * NW;
  const Prim<DIM> s = prim<DIM>(W, p.NR);
  int N = 0;
  double mk = 0.0;
  if (!prim_ok(s)) {
    atomicOr(st.flags, kFlagInvalid);
    st.tau[i] = 1.0;
    st.E[i] = 0.0;
    st.hvalid[i] = 0;
  } else {
    const double tau = relax_time(p, case_val(g, case_of(g, i), kCaseMu, p.mu_ref), s.rho, s.T);
    const double E = p.wave_only ? 0.0 : exp(-(st.dt[i] / tau));
    st.tau[i] = tau;
    st.E[i] = E;
    st.tdt[i] = make_double2(tau, st.dt[i]);
    double Wh[NW];
    const double vol = g.vol[i];
#pragma unroll
    for (int q = 0; q < NW; ++q) {
      Wh[q] = W[q] - st.Sret[i * NW + q] / vol;
      st.Wh[i * NW + q] = Wh[q];
    }
    const Prim<DIM> h = prim<DIM>(Wh, p.NR);
    const bool hv = prim_ok(h);
    st.hvalid[i] = hv ? 1 : 0;
    if (p.Pr != 1.0) {
      // heat flux of the retained particles relative to U_i (Eq. (5)):
      // Q_a = 1/2 sum m (u - U)_a |u - U|^2 expanded in raw moments
      const double *Sr = st.Sret + i * NW;
      const double *Mr = st.Mraw + i * 5;
      const double Ux = s.ux, Uy = s.uy;
      const double m0 = Sr[0], mx = Sr[1], my = DIM == 2 ? Sr[2] : 0.0, mq = 2.0 * Sr[NW - 1];
      const double UU = Ux * Ux + Uy * Uy;
      const double PxU = Mr[2] * Ux + Mr[3] * Uy, PyU = Mr[3] * Ux + Mr[4] * Uy;
      const double mU = mx * Ux + my * Uy;
      const double Qx = 0.5 * ((((Mr[0] - 2.0 * PxU) + UU * mx) - Ux * mq) + (2.0 * Ux * mU - Ux * UU * m0));
      const double Qy = 0.5 * ((((Mr[1] - 2.0 * PyU) + UU * my) - Uy * mq) + (2.0 * Uy * mU - Uy * UU * m0));
      if (hv) {
        // acceptance-rejection constants of the Shakhov target for the
        // cell's new particles: proposal = Maxwellian of W^h, target
        // parameters = U, T, p and heat flux of the cell total
        double *a = st.ar + i * kArN;
        const double sh3 = s.rho * p.R * s.T, sh4 = Qx / vol, sh5 = Qy / vol;
        const double sig = sqrt(p.R * h.T);
        const double RT = p.R * s.T;
        const double cmax = 6.0 * sig;
        const double du = sqrt((h.ux - s.ux) * (h.ux - s.ux) + (h.uy - s.uy) * (h.uy - s.uy));
        const double cb = cmax + du;
        const double qn = sqrt(sh4 * sh4 + sh5 * sh5);
        const double w = cb * cb / RT - 5.0;
        a[kArUhx] = h.ux;
        a[kArUhy] = h.uy;
        a[kArSig] = sig;
        a[kArCmax] = cmax;
        a[kArRT] = RT;
        a[kArBnd] = 1.0 + (fabs(1.0 - p.Pr) * qn * cb * (w > 5.0 ? w : 5.0)) / (5.0 * sh3 * RT);
        a[kArUx] = s.ux;
        a[kArUy] = s.uy;
        a[kArP] = sh3;
        a[kArQx] = sh4;
        a[kArQy] = sh5;
      }
    }
    if (hv) {
      const double rho_hp = Wh[0] * E;
      if (rho_hp > 0.0) {
        const double ratio = rho_hp / W[0];
        const double Nd = ceil(ratio * static_cast<double>(p.n_ref));
        if (Nd > 1048575.0) {
          atomicOr(st.flags, kFlagOverflow);
        } else {
          N = static_cast<int>(Nd);
          mk = (rho_hp * vol) / static_cast<double>(N);
        }
      }
    }
  }
  st.ncount[i] = N;
  st.mnew[i] = mk;
}

// Ghost states of boundary faces (both sides use dt_i, Sec. IV.B): far field
// fixed, outflow = copy of W_i, symmetry = mirror of W_i and W^h_i.  For far
// field and outflow, the injection slab of depth dt_i (U_in + 6 sqrt(R T_g))
// behind the face and its particle count relative to Omega_i.
template <int DIM>
__global__ void k_ghost_prep(Geo g, Params p, State st) {
  constexpr int NW = DIM + 2;
  const int64_t b = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (b >= g.nb || *st.halt) return;
  const int i = g.bcell[b];
  const int ty = g.btype[b];
  const double4 f = g.lfn[static_cast<int64_t>(i) * g.NV + g.bk[b]];
  double W[4] = {0, 0, 0, 0}, Wh[4] = {0, 0, 0, 0};
  int hv = 0;
  double tau = st.tau[i];
  if (ty == kBcFarfield) {
    const double *d = g.bdata + 8 * b;
    const double ke = 0.5 * d[0] * (d[1] * d[1] + (DIM == 2 ? d[2] * d[2] : 0.0));
    W[0] = d[0];
    W[1] = d[0] * d[1];
    if (DIM == 2) W[2] = d[0] * d[2];
    W[DIM + 1] = ke + 0.5 * p.Nd * d[0] * p.R * d[3];
    for (int q = 0; q < NW; ++q) Wh[q] = W[q];
    hv = 1;
    tau = relax_time(p, case_val(g, case_of(g, i), kCaseMu, p.mu_ref), d[0], d[3]);
  } else if (ty == kBcOutflow) {
    for (int q = 0; q < NW; ++q) Wh[q] = W[q] = st.W[static_cast<int64_t>(i) * NW + q];
    hv = 1;
  } else if (ty == kBcSymmetry || ty == kBcMaxwell) {
    // mirror state (also the specular part of a Maxwell wall)
    for (int q = 0; q < NW; ++q) {
      W[q] = st.W[static_cast<int64_t>(i) * NW + q];
      Wh[q] = st.Wh[static_cast<int64_t>(i) * NW + q];
    }
    if (DIM == 2) {
      const double mn = W[1] * f.x + W[2] * f.y;
      const double w1 = W[1] - 2.0 * mn * f.x, w2 = W[2] - 2.0 * mn * f.y;
      W[1] = w1;
      W[2] = w2;
      const double hn = Wh[1] * f.x + Wh[2] * f.y;
      const double h1 = Wh[1] - 2.0 * hn * f.x, h2 = Wh[2] - 2.0 * hn * f.y;
      Wh[1] = h1;
      Wh[2] = h2;
    } else {
      W[1] = -W[1];
      Wh[1] = -Wh[1];
    }
    hv = st.hvalid[i];
  }
  const double dti = st.dt[i];
  const double E = p.wave_only ? 0.0 : exp(-(dti / tau));
  for (int q = 0; q < NW; ++q) {
    st.gW[b * NW + q] = W[q];
    st.gWh[b * NW + q] = Wh[q];
  }
  st.gtau[b] = tau;
  st.ghvalid[b] = hv;
  int N = 0;
  double mk = 0.0, depth = 0.0;
  if (ty == kBcFarfield || ty == kBcOutflow) {
    const Prim<DIM> s = prim<DIM>(W, p.NR);
    const double Uin = -(DIM == 2 ? s.ux * f.x + s.uy * f.y : s.ux * f.x);
    depth = dti * (Uin + 6.0 * sqrt(p.R * s.T));
    if (depth > 0.0) {
      const double Mslab = s.rho * E * depth * g.lfs[static_cast<int64_t>(i) * g.NV + g.bk[b]];
      if (Mslab > 0.0) {
        const double Nd = ceil((Mslab / (s.rho * g.vol[i])) * static_cast<double>(p.n_ref));
        if (Nd > 1048575.0) {
          atomicOr(st.flags, kFlagOverflow);
        } else {
          N = static_cast<int>(Nd);
          mk = Mslab / static_cast<double>(N);
        }
      }
    }
  }
  st.ncount[g.nc + b] = N;
  st.mnew[g.nc + b] = mk;
  st.gdepth[b] = depth;
}

// ---------------------------------------------------------------------------
// Exclusive scan of int counts into int64 offsets in two launches: block
// scans with their sums, then an add pass in which every block sums the block
// sums before it.  kScanBlock elements per block.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t block_excl_scan(int64_t v, int64_t *sh, int64_t &total) {
  // sh: blockDim.x entries; Hillis-Steele on wavefront sums
  const int t = threadIdx.x;
  const int lane = t & 63, w = t >> 6;
  int64_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh[w] = x;
  __syncthreads();
  const int nwaves = blockDim.x >> 6;
  if (t == 0) {
    int64_t acc = 0;
    for (int k = 0; k < nwaves; ++k) {
      const int64_t s = sh[k];
      sh[k] = acc;
      acc += s;
    }
    sh[nwaves] = acc;
  }
  __syncthreads();
  total = sh[nwaves];
  const int64_t r = sh[w] + x - v;
  __syncthreads();
  return r;
}

__global__ void k_scan_blocks(const int *__restrict__ in, int64_t n, int64_t *__restrict__ out,
                              int64_t *__restrict__ bsum, const int *__restrict__ halt) {
  __shared__ int64_t sh[kScanBlock / 64 + 1];
  if (*halt) return;
  const int64_t i = blockIdx.x * static_cast<int64_t>(kScanBlock) + threadIdx.x;
  const int64_t v = i < n ? in[i] : 0;
  int64_t total;
  const int64_t r = block_excl_scan(v, sh, total);
  if (i < n) out[i] = r;
  if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}


// Adds to each block's scan the sum of the block sums before it (each block
// sums them itself: there are few) and writes the total to out[n].  Also
// copies the first n results to out2 when given (the scatter's cursors).
__global__ void k_scan_add(int64_t *__restrict__ out, int64_t n, const int64_t *__restrict__ bsum,
                           const int *__restrict__ halt, int64_t *__restrict__ out2) {
  __shared__ int64_t sh[kScanBlock / 64 + 1];
  if (*halt) return;  // uniform: nothing changes halt during the scan
  int64_t part = 0;
  for (int64_t k = threadIdx.x; k < static_cast<int64_t>(blockIdx.x); k += blockDim.x) part += bsum[k];
  int64_t carry;
  (void)block_excl_scan(part, sh, carry);
  const int64_t i = blockIdx.x * static_cast<int64_t>(kScanBlock) + threadIdx.x;
  if (i < n) {
    const int64_t v = out[i] + carry;
    out[i] = v;
    if (out2) out2[i] = v;
  }
  if (i == n) out[n] = carry + bsum[blockIdx.x];
}

// ---------------------------------------------------------------------------
// a3: resampling.  One wavefront per cell draws its N new particles:
// position uniform in the cell, deviation z from the Maxwellian of W^h (with
// Shakhov acceptance-rejection when Pr != 1), t_f = dt_i, pid = n<<44|i<<20|j.
// For N >= 2 the set is shifted to zero mean and scaled so that it carries
// exactly the momentum and thermal energy of W^hp (Eq. (25)).  The kernel
// also writes W^{p,-} Omega = W^p Omega + the new particles' tally.
// ---------------------------------------------------------------------------
template <int DIM>
__device__ __forceinline__ void sample_position(const Geo &g, int64_t cell, uint64_t seed, uint64_t pid,
                                                int64_t step, double &x, double &y) {
  double e0, e1, e2, e3;
  rng2(seed, pid, step, kPos, 0, e0, e1);
  const double2 *v = g.cverts + cell * g.NV;
  if (DIM == 1) {
    const double xl = v[0].x, xr = v[1].x;
    x = xl + e0 * (xr - xl);
    y = 0.0;
    return;
  }
  rng2(seed, pid, step, kPos, 1, e2, e3);
  const int nv = g.nv[cell];
  const double x0 = v[0].x, y0 = v[0].y;
  const double target = e0 * g.vol[cell];
  double acc = 0.0;
  int t = 0;
  for (t = 0; t + 2 < nv; ++t) {
    const double xa = v[t + 1].x, ya = v[t + 1].y, xb = v[t + 2].x, yb = v[t + 2].y;
    acc += 0.5 * ((xa - x0) * (yb - y0) - (xb - x0) * (ya - y0));
    if (target < acc) break;
  }
  if (t + 2 >= nv) t = nv - 3;
  const double xa = v[t + 1].x, ya = v[t + 1].y, xb = v[t + 2].x, yb = v[t + 2].y;
  double b1 = e1, b2 = e2;
  if (b1 + b2 > 1.0) {
    b1 = 1.0 - b1;
    b2 = 1.0 - b2;
  }
  x = (x0 + b1 * (xa - x0)) + b2 * (xb - x0);
  y = (y0 + b1 * (ya - y0)) + b2 * (yb - y0);
}

// One acceptance-rejection attempt `att` for the Shakhov target (Eq. (4))
// against the Maxwellian of W^h (table a of the cell, from cell_prep):
// draws z (calls 2 att, 2 att + 1); returns 0 if the deviation lies beyond
// the 6 sigma cut, 1 if inside but rejected, 2 if accepted (probability
// (1 + phi) / B).  z is set in every case.
template <int DIM>
__device__ __forceinline__ int shakhov_attempt(const Params &p, const double *a, uint64_t seed, uint64_t pid,
                                               int64_t step, uint32_t att, double z[3]) {
  gauss3(seed, pid, step, kVel, 2 * att, z);
  const double sig = a[kArSig];
  const double dz = sqrt(z[0] * z[0] + z[1] * z[1] + z[2] * z[2]) * sig;
  if (dz > a[kArCmax]) return 0;
  double ea, eb;
  rng2(seed, pid, step, kShakhov, att, ea, eb);
  const double RT = a[kArRT];
  const double cx = (a[kArUhx] + sig * z[0]) - a[kArUx], cy = (a[kArUhy] + sig * z[1]) - a[kArUy];
  const double cz = sig * z[2];
  const double c2 = cx * cx + cy * cy + cz * cz;
  const double cq = DIM == 2 ? cx * a[kArQx] + cy * a[kArQy] : cx * a[kArQx];
  const double phi = ((1.0 - p.Pr) * cq) / (5.0 * a[kArP] * RT) * (c2 / RT - 5.0);
  return ea * a[kArBnd] <= 1.0 + phi ? 2 : 1;
}

// Draw pass: one thread per new particle of the interior cells.  The birth
// cell i is the last cell with noff[i] <= k (binary search over the exclusive
// scan of the counts), j = k - noff[i].  Writes the position, the raw
// deviation z (in the velocity slots), pid, cell and mass.
template <int DIM, class R>
__device__ __forceinline__ void sample_draw_one(const Geo &g, const Params &p, const State &st, const StoreT<R> &out,
                                                int64_t n_ret, int64_t step, int64_t k) {
  constexpr int NW = DIM + 2;
  int64_t lo = 0, hi = g.nc;
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (st.noff[mid] <= k) lo = mid;
    else hi = mid;
  }
  const int64_t i = lo;
  const int64_t j = k - st.noff[i];
  const int cs = case_of(g, i);
  const uint64_t seed = case_seed(g, p, cs);
  const int64_t li = g.ccase ? i - g.case_cell[cs] : i;  // cell within its case
  const uint64_t pid = (static_cast<uint64_t>(step) << 44) | (static_cast<uint64_t>(li) << 20) |
                       static_cast<uint64_t>(j);
  double x, y;
  sample_position<DIM>(g, i, seed, pid, step, x, y);
  const int64_t o = n_ret + k;
  store_position<DIM, R>(g, out, o, i, x, y);
  if (p.Pr == 1.0) {
    // Maxwellian of W^h; with Pr != 1 k_sample_shakhov draws z
    double z[3];
    gauss3(seed, pid, step, kVel, 0, z);
    out.ux[o] = static_cast<R>(z[0]);
    out.uy[o] = static_cast<R>(z[1]);
    out.uz[o] = static_cast<R>(z[2]);
  }
  if (out.ei) out.ei[o] = static_cast<R>(internal_eta(seed, pid, step, 0, p.D));  // eta; scaled in k_sample_match
  out.pid[o] = pid;
  out.cell[o] = static_cast<int>(i);
  out.m[o] = st.mnew[i];
  (void)NW;
}

template <int DIM, class R>
__global__ void __launch_bounds__(256) k_sample_draw(Geo g, Params p, State st, StoreT<R> out, int64_t cap) {
  if (*st.halt) return;
  const int64_t n_ret = st.roff[g.nc], n_cellnew = st.noff[g.nc], step = *st.dstep;
  const int64_t k = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (k < n_cellnew && n_ret + k < cap) sample_draw_one<DIM, R>(g, p, st, out, n_ret, step, k);
}

// Shakhov deviations of the new particles (Pr != 1).  The result is that of
// the sequential rule: the lowest accepted attempt of 0..63; if none is
// accepted (a fallback, counted), the lowest attempt inside the 6 sigma cut,
// or z = 0 if there is none.
// An attempt is a long dependent chain (Philox, logarithms, sine/cosine) and
// the number of attempts varies widely (about the acceptance bound B; all
// 64 in near-vacuum cells where B is huge), so work is spread over lanes:
//  1. a wavefront takes 64/K particles, K lanes each (K = `lanes`, a tuning
//     parameter in {1, 2, 4, 8, 16}); the K lanes of a particle evaluate
//     attempts 0..K-1 at once and keep the lowest accepted one;
//  2. the particles not yet accepted are finished in the same way with L
//     lanes each on attempts K, K + L, ...: L = 64 / n rounded down to a
//     power of two for n remaining particles, at least 8, so that up to
//     eight remaining particles share one round, and a lone near-vacuum
//     particle, which needs every attempt, gets all 64 lanes.
// More lanes per particle means more wavefronts in flight to hide latency.
template <int DIM, class R>
__global__ void __launch_bounds__(256) k_sample_shakhov(Geo g, Params p, State st, StoreT<R> out, int64_t cap,
                                                        uint32_t lanes) {
  if (*st.halt) return;
  const int64_t n_ret = st.roff[g.nc], step = *st.dstep;
  int64_t end = st.noff[g.nc];
  if (end > cap - n_ret) end = cap - n_ret;
  const int K1 = static_cast<int>(lanes), P1 = 64 / K1;
  const int64_t base = ((blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x) >> 6) * P1;
  if (base >= end) return;  // whole wavefront
  const int lane = lane_id();
  const int g1 = lane / K1, s1 = lane % K1;
  const int64_t kp = base + g1;
  const bool act = kp < end;
  uint64_t pid = 0, seed = 0;
  int cell = 0;
  if (act) {
    pid = out.pid[n_ret + kp];
    cell = out.cell[n_ret + kp];
    seed = case_seed(g, p, case_of(g, cell));
  }
  int ncapped = 0;
  // phase 1
  {
    double z[3] = {0.0, 0.0, 0.0};
    const int res = act ? shakhov_attempt<DIM>(p, st.ar + static_cast<int64_t>(cell) * kArN, seed, pid, step,
                                               static_cast<uint32_t>(s1), z)
                        : 0;
    const uint64_t gmask = K1 == 64 ? ~0ull : ((1ull << K1) - 1ull);
    const uint64_t seg = (__ballot(res == 2) >> (g1 * K1)) & gmask;
    const uint64_t segin = (__ballot(res >= 1) >> (g1 * K1)) & gmask;
    // lowest attempt inside the cut so far (phase 1 attempt = lane in group)
    const int first_in = segin ? __ffsll(static_cast<long long>(segin)) - 1 : -1;
    if (act && seg != 0 && s1 == __ffsll(static_cast<long long>(seg)) - 1) {
      const int64_t o = n_ret + kp;
      out.ux[o] = static_cast<R>(z[0]);
      out.uy[o] = static_cast<R>(z[1]);
      out.uz[o] = static_cast<R>(z[2]);
    }
    // one bit per particle still to do, at the first lane of its group
    const uint64_t open = __ballot(act && seg == 0 && s1 == 0);
    if (!open) return;
    uint64_t hard = open;
    while (hard) {
      const int nh = __popcll(hard);
      // lanes per particle (uniform): 64 / nh rounded down to a power of
      // two, at least 8 (a round of many particles with few lanes each
      // would idle lanes on the slowest ones)
      const int L = nh == 1 ? 64 : nh == 2 ? 32 : nh <= 4 ? 16 : 8;
      const int grp = lane / L, sl = lane % L;
      const uint64_t segm = L == 64 ? ~0ull : ((1ull << L) - 1ull);
      // this group's particle: the grp-th remaining one, if any
      uint64_t h = hard;
      for (int q = 0; q < grp && h; ++q) h &= h - 1;
      const int src = h ? __ffsll(static_cast<long long>(h)) - 1 : -1;
      for (int q = 0; q < 64 / L && hard; ++q) hard &= hard - 1;  // the chunk taken
      const int sv = src < 0 ? 0 : src;
      const uint64_t gpid = __shfl(pid, sv, 64);
      const uint64_t gseed = __shfl(seed, sv, 64);
      const int gcell = __shfl(cell, sv, 64);
      const int64_t gk = __shfl(kp, sv, 64);
      int gin = __shfl(first_in, sv, 64);
      const double *tab = st.ar + static_cast<int64_t>(gcell) * kArN;
      bool gdone = src < 0;
      uint32_t a = static_cast<uint32_t>(K1);
      while (__ballot(!gdone)) {
        const uint32_t att = a + static_cast<uint32_t>(sl);
        double w[3] = {0.0, 0.0, 0.0};
        int res2 = 0;
        if (!gdone && att < 64) res2 = shakhov_attempt<DIM>(p, tab, gseed, gpid, step, att, w);
        const uint64_t sg = (__ballot(res2 == 2) >> (grp * L)) & segm;
        const uint64_t sgin = (__ballot(res2 >= 1) >> (grp * L)) & segm;
        if (!gdone) {
          if (gin < 0 && sgin != 0) gin = static_cast<int>(a) + __ffsll(static_cast<long long>(sgin)) - 1;
          if (sg != 0) {
            if (sl == __ffsll(static_cast<long long>(sg)) - 1) {
              const int64_t d = n_ret + gk;
              out.ux[d] = static_cast<R>(w[0]);
              out.uy[d] = static_cast<R>(w[1]);
              out.uz[d] = static_cast<R>(w[2]);
            }
            gdone = true;
          } else if (a + static_cast<uint32_t>(L) >= 64) {
            // no attempt accepted: the first draw inside the cut, else 0
            if (sl == 0) {
              double zf[3] = {0.0, 0.0, 0.0};
              if (gin >= 0) gauss3(gseed, gpid, step, kVel, 2 * static_cast<uint32_t>(gin), zf);
              const int64_t d = n_ret + gk;
              out.ux[d] = static_cast<R>(zf[0]);
              out.uy[d] = static_cast<R>(zf[1]);
              out.uz[d] = static_cast<R>(zf[2]);
              ++ncapped;
            }
            gdone = true;
          } else {
            a += static_cast<uint32_t>(L);
          }
        }
      }
    }
  }
  const uint64_t mc = __ballot(ncapped > 0);
  if (mc) {
    // at most one capped particle per lane per round; sum the lanes' counts
    int tot = ncapped;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) tot += __shfl_xor(tot, o, 64);
    if (lane == 0)
      atomicAdd(reinterpret_cast<unsigned long long *>(&st.stats[(blockIdx.x % kStatSlots) * kStatN + kStatCapped]),
                static_cast<unsigned long long>(tot));
  }
}

// Moment-matching pass: sixteen lanes per cell (four cells per wavefront:
// a cell draws about twenty new particles in the benchmark flow) over its
// new particles.  For
// N >= 2 the deviations are shifted to zero mean and scaled so that the set
// carries exactly the momentum and thermal energy of W^hp (Eq. (25)):
// u = U^h + sqrt(R T^h) ((z - zbar) alpha), alpha = sqrt(3 N / sum |z - zbar|^2).
// Also W^{p,-} Omega = W^p Omega + the new set's tally (Eq. (30)), rounded
// once from the exact chunks of both.  Every reduction stays within the
// cell's sixteen lanes (exchanges at distance 8, 4, 2, 1).
constexpr int kMatchLanes = 16;

__device__ __forceinline__ double seg_sum(double v) {
#pragma unroll
  for (int o = kMatchLanes / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// One halving exchange at distance O: of 2H values, a lane keeps the half
// its bit O selects and adds the partner's copy of it.
template <int H, int O>
__device__ __forceinline__ void seg_halve(double (&v)[32]) {
  const bool hi = (lane_id() & O) != 0;
#pragma unroll
  for (int j = 0; j < H; ++j) {
    const double send = hi ? v[j] : v[j + H];
    const double keep = hi ? v[j + H] : v[j];
    v[j] = keep + __shfl_xor(send, O, 64);
  }
}

// Totals of 32 values over a cell's sixteen lanes: on return, lane r of the
// segment holds the totals of values 2r (in v[0]) and 2r + 1 (in v[1]).
__device__ __forceinline__ void seg_spread32(double (&v)[32]) {
  seg_halve<16, 8>(v);
  seg_halve<8, 4>(v);
  seg_halve<4, 2>(v);
  seg_halve<2, 1>(v);
}

template <int DIM, class R>
__global__ void __launch_bounds__(256) k_sample_match(Geo g, Params p, State st, StoreT<R> out, int64_t cap) {
  constexpr int NW = DIM + 2;
  constexpr int NLT = kTallyLimbs;
  static_assert(NLT == 6 && NW * NLT <= 32, "the writer layout assumes six chunks per component");
  const int64_t i = (blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x) / kMatchLanes;
  // a segment (one cell) returns as a whole; reductions stay inside segments
  if (i >= g.nc || *st.halt) return;
  const int sl = lane_id() % kMatchLanes;
  // component q is gathered by segment lane 3 q (its chunks sit at lanes 3 q,
  // 3 q + 1 and 3 q + 2, two each)
  const int q = sl / 3;
  const bool writer = sl % 3 == 0 && q < NW;
  // the retained tally's exact chunks, loaded early (independent of the rest)
  double xr[NLT];
#pragma unroll
  for (int jj = 0; jj < NLT; ++jj) xr[jj] = writer ? st.Xret[(i * NW + q) * NLT + jj] : 0.0;
  const int64_t n_ret = st.roff[g.nc];
  const int N = n_ret + st.noff[i] + st.ncount[i] <= cap ? st.ncount[i] : 0;
  // chunks of the new set's tally: value q * kTallyLimbs + j = chunk j of component q
  double xc[32];
#pragma unroll
  for (int k = 0; k < 32; ++k) xc[k] = 0.0;
  bool ok = true;
  if (N > 0) {
    const int64_t base = n_ret + st.noff[i];
    const Prim<DIM> h = prim<DIM>(st.Wh + i * NW, p.NR);
    const double sig = sqrt(p.R * h.T);
    const double mk = st.mnew[i];
    // the first sixteen particles' deviations stay in registers across the passes
    const bool own = sl < N;
    const double z0 = own ? static_cast<double>(out.ux[base + sl]) : 0.0;
    const double z1 = own ? static_cast<double>(out.uy[base + sl]) : 0.0;
    const double z2 = own ? static_cast<double>(out.uz[base + sl]) : 0.0;
    const double e0 = own && out.ei ? static_cast<double>(out.ei[base + sl]) : 0.0;
    double zm[3] = {0.0, 0.0, 0.0};
    double alpha = 1.0, beta = 1.0;
    if (N >= 2) {
      double zs[3] = {z0, z1, z2}, es = e0;
      for (int j = sl + kMatchLanes; j < N; j += kMatchLanes) {
        zs[0] += out.ux[base + j];
        zs[1] += out.uy[base + j];
        zs[2] += out.uz[base + j];
        if (out.ei) es += out.ei[base + j];
      }
#pragma unroll
      for (int d = 0; d < 3; ++d) zm[d] = seg_sum(zs[d]) / static_cast<double>(N);
      // the internal energies are scaled to carry exactly D R T^h / 2 per unit mass
      if (out.ei) beta = (0.5 * static_cast<double>(p.D) * static_cast<double>(N)) / seg_sum(es);
      double S = 0.0;
      if (own) {
        const double a0 = z0 - zm[0], a1 = z1 - zm[1], a2 = z2 - zm[2];
        S = a0 * a0 + a1 * a1 + a2 * a2;
      }
      for (int j = sl + kMatchLanes; j < N; j += kMatchLanes) {
        const double a0 = out.ux[base + j] - zm[0], a1 = out.uy[base + j] - zm[1], a2 = out.uz[base + j] - zm[2];
        S += a0 * a0 + a1 * a1 + a2 * a2;
      }
      S = seg_sum(S);
      alpha = sqrt((3.0 * static_cast<double>(N)) / S);
    }
    for (int j = sl; j < N; j += kMatchLanes) {
      const int64_t k = base + j;
      const bool first = j == sl;
      const double y0 = first ? z0 : static_cast<double>(out.ux[k]);
      const double y1 = first ? z1 : static_cast<double>(out.uy[k]);
      const double y2 = first ? z2 : static_cast<double>(out.uz[k]);
      const double w0 = (y0 - zm[0]) * alpha, w1 = (y1 - zm[1]) * alpha, w2 = (y2 - zm[2]) * alpha;
      // the stored velocities (rounded in the FP32 store) enter the tally
      const R r0 = static_cast<R>(h.ux + sig * w0), r1 = static_cast<R>(h.uy + sig * w1), r2 = static_cast<R>(sig * w2);
      out.ux[k] = r0;
      out.uy[k] = r1;
      out.uz[k] = r2;
      double ei = 0.0;
      if (out.ei) {
        const double y3 = first ? e0 : static_cast<double>(out.ei[k]);
        const R re = static_cast<R>((p.R * h.T) * (beta * y3));
        out.ei[k] = re;
        ei = re;
      }
      const double u0 = r0, u1 = r1, u2 = r2;
      const double en = 0.5 * (u0 * u0 + u1 * u1 + u2 * u2) + ei;
      double t[NW];
      t[0] = mk;
      t[1] = mk * u0;
      if (DIM == 2) t[2] = mk * u1;
      t[NW - 1] = mk * en;
#pragma unroll
      for (int c = 0; c < NW; ++c) {
        double ch[NLT];
        ok = xs_split<NLT>(t[c], p.xw, ch) && ok;
#pragma unroll
        for (int jj = 0; jj < NLT; ++jj) xc[c * NLT + jj] += ch[jj];
      }
    }
  }
  if (!ok) {
    atomicOr(st.flags, kFlagRange);
    atomicOr(st.halt, 1);
  }
  double L[NLT];
  if (N > 0) {
    seg_spread32(xc);
    const double b0 = __shfl(xc[0], lane_id() + 1, 64), b1 = __shfl(xc[1], lane_id() + 1, 64);
    const double c0 = __shfl(xc[0], lane_id() + 2, 64), c1 = __shfl(xc[1], lane_id() + 2, 64);
    L[0] = xc[0] + xr[0];
    L[1] = xc[1] + xr[1];
    L[2] = b0 + xr[2];
    L[3] = b1 + xr[3];
    L[4] = c0 + xr[4];
    L[5] = c1 + xr[5];
  } else {
#pragma unroll
    for (int jj = 0; jj < NLT; ++jj) L[jj] = xr[jj];
  }
  if (writer) st.Sm[i * NW + q] = xs_round<NLT>(L, p.xw);
}

// Ghost injection: one wavefront per far-field/outflow face samples its slab;
// particles whose straight flight reaches the face within dt_i enter cell i
// at the crossing point (tangential position wrapped along the face) with the
// remaining time.  Entering particles are compacted by ballot and appended.
template <int DIM, class R>
__global__ void __launch_bounds__(256) k_sample_ghosts(Geo g, Params p, State st, StoreT<R> out, int64_t cap) {
  constexpr int NW = DIM + 2;
  const int64_t b = (blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x) >> 6;
  if (b >= g.nb || *st.halt) return;
  const int64_t gbase = st.roff[g.nc] + st.noff[g.nc], step = *st.dstep;
  const int N = st.ncount[g.nc + b];
  if (N == 0) return;
  const int lane = lane_id();
  const int i = g.bcell[b];
  const int kf = g.bk[b];
  const double4 f = g.lfn[static_cast<int64_t>(i) * g.NV + kf];
  const Prim<DIM> s = prim<DIM>(st.gW + b * NW, p.NR);
  const double sg = sqrt(p.R * s.T);
  const double depth = st.gdepth[b];
  const double mk = st.mnew[g.nc + b];
  const double dti = st.dt[i];
  const double2 *v = g.cverts + static_cast<int64_t>(i) * g.NV;
  const int nv = DIM == 2 ? g.nv[i] : 2;
  // birth "cell" of an injected particle: the face after the case's cells
  const int cs = case_of(g, i);
  const uint64_t seed = case_seed(g, p, cs);
  const int64_t gid = g.ccase ? (g.case_cell[cs + 1] - g.case_cell[cs]) + (b - g.case_bface[cs]) : g.nc + b;
  const double xa = DIM == 2 ? v[kf].x : v[kf].x, ya = DIM == 2 ? v[kf].y : 0.0;
  const double xb = DIM == 2 ? v[(kf + 1) % nv].x : 0.0, yb = DIM == 2 ? v[(kf + 1) % nv].y : 0.0;
  for (int j0 = 0; j0 < N; j0 += 64) {
    const int j = j0 + lane;
    bool enter = false;
    double px = 0, py = 0, u0 = 0, u1 = 0, u2 = 0, tr = 0;
    uint64_t pid = 0;
    if (j < N) {
      pid = (static_cast<uint64_t>(step) << 44) | (static_cast<uint64_t>(gid) << 20) | static_cast<uint64_t>(j);
      double e0, e1, z[3];
      rng2(seed, pid, step, kPos, 0, e0, e1);
      gauss3(seed, pid, step, kVel, 0, z);
      u0 = s.ux + sg * z[0];
      u1 = s.uy + sg * z[1];
      u2 = sg * z[2];
      const double vin = -(DIM == 2 ? u0 * f.x + u1 * f.y : u0 * f.x);
      if (vin > 0.0) {
        const double tc = (e0 * depth) / vin;
        if (tc < dti) {
          enter = true;
          tr = dti - tc;
          if (DIM == 2) {
            const double sface = g.lfs[static_cast<int64_t>(i) * g.NV + kf];
            const double ut = u1 * f.x - u0 * f.y;
            double a = e1 * sface + ut * tc;
            a = a - sface * floor(a / sface);
            const double w = a / sface;
            px = xa + w * (xb - xa);
            py = ya + w * (yb - ya);
          } else {
            px = xa;
          }
        }
      }
    }
    const uint64_t mask = __ballot(enter);
    int64_t pos = 0;
    if (lane == 0 && mask) pos = atomicAdd(reinterpret_cast<unsigned long long *>(st.nghost),
                                           static_cast<unsigned long long>(__popcll(mask)));
    pos = __shfl(pos, 0, 64);
    if (enter && gbase + pos + popc_below(mask) < cap) {
      const int64_t r = pos + popc_below(mask);
      const int64_t k = gbase + r;
      store_position<DIM, R>(g, out, k, i, px, py);
      out.ux[k] = static_cast<R>(u0);
      out.uy[k] = static_cast<R>(u1);
      out.uz[k] = static_cast<R>(u2);
      if (out.ei) out.ei[k] = static_cast<R>((p.R * s.T) * internal_eta(seed, pid, step, 0, p.D));
      out.m[k] = mk;
      out.pid[k] = pid;
      out.cell[k] = i;
      st.tghost[r] = tr;
    }
  }
}

// ---------------------------------------------------------------------------
// a4 + a6 + a7 (tally part): one thread per particle.
// Free-transport time of retained particles (Eq. (51)); tracking with the
// crossing scaling m <- m r, t <- (t - t_e) r, r = dt_R/dt_L (Eqs. (41), (52));
// exit face = smallest t_e = (c_e - n_e.x)/(u.n_e) over u.n_e > 0 (clamped at
// 0, ties to the lowest local index), crossing iff t_e < t; far field and
// outflow remove, symmetry reflects specularly, diffuse walls re-emit
// (normal speed sqrt(-2 R T_w ln e), WALL draws 2h, 2h+1 for the h-th hit).
// Then W^{p,+} Omega over every particle ending inside (Eq. (30)), the next
// step's W^p Omega and counts over the kept (non-collided) ones.
// ---------------------------------------------------------------------------
template <class R> struct Face;
template <> struct Face<double> { using type = double4; };
template <> struct Face<float> { using type = float4; };

// Face data of local face l for tracking: (n_x, n_y, offset c, ratio).  The
// FP32 table's offset is relative to the cell's anchor.
template <class R>
__device__ __forceinline__ typename Face<R>::type load_face(const Geo &g, int64_t l) {
  if constexpr (IsF32<R>::value) return g.lfn32[l];
  else return g.lfn[l];
}

// Particle impulse on a wall face: exact chunks (window xw) of
// m (u_before - u_after) (x, y) and of the energy given up, added
// atomically (order-independent).
__device__ __forceinline__ void wall_impulse(const Params &p, const State &st, int bf, double ix, double iy, double ie) {
  constexpr int NLT = kTallyLimbs;
  const double v[3] = {ix, iy, ie};
  bool ok = true;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    double c[NLT];
    ok = xs_split<NLT>(v[q], p.xw, c) && ok;
#pragma unroll
    for (int j = 0; j < NLT; ++j)
      if (c[j] != 0.0) atomicAdd(&st.wimp[(3 * bf + q) * NLT + j], c[j]);
  }
  if (!ok) {
    atomicOr(st.flags, kFlagRange);
    atomicOr(st.halt, 1);
  }
}

template <int DIM, int NV, class R, int FEAT>
__device__ __forceinline__ void transport_one(const Geo &g, const Params &p, const State &st, const StoreT<R> &s,
                                              const StoreT<R> &tw, int64_t n_ret, int64_t gbase, int64_t n_total,
                                              int64_t step, int64_t k) {
  constexpr int NW = DIM + 2;
  constexpr bool F32 = IsF32<R>::value;
  using F4 = typename Face<R>::type;
  const bool active = k < n_total;
  int cell = -1;
  bool exited = false, collide = false;
  R x = 0, y = 0, u0 = 0, u1 = 0, u2 = 0, ei = 0;
  double m = 0;
  if (active) {
    cell = s.cell[k];
    x = s.x[k];
    y = DIM == 2 ? s.y[k] : R(0);
    u0 = s.ux[k];
    u1 = s.uy[k];
    u2 = s.uz[k];
    if constexpr ((FEAT & kFeatEi) != 0) ei = s.ei[k];
    m = s.m[k];
    const uint64_t pid = s.pid[k];
    const uint64_t seed = case_seed(g, p, case_of(g, cell));
    // the cell's face normals, offsets and neighbours, loaded together on
    // entering a cell and again after a reflection (so that they are dead in
    // the reflection code); a face's ratio is loaded when it is crossed
    R Fx[NV], Fy[NV], Fz[NV];
    int nbr[NV];
    const double2 td = st.tdt[cell];
    auto load_cell = [&](int c) {
#pragma unroll
      for (int kk = 0; kk < NV; ++kk) {
        const F4 f = load_face<R>(g, static_cast<int64_t>(c) * NV + kk);
        Fx[kk] = f.x;
        Fy[kk] = f.y;
        Fz[kk] = f.z;
        nbr[kk] = g.lnb[static_cast<int64_t>(c) * NV + kk];
      }
    };
    load_cell(cell);
    R t;
    if (k < n_ret) {
      double e0, e1;
      rng2(seed, pid, step, kFree, 0, e0, e1);
      const double sfree = -td.x * log(e0);
      collide = sfree < td.y;
      t = static_cast<R>(collide ? sfree : td.y);
    } else if (k < gbase) {
      t = static_cast<R>(td.y);
    } else {
      t = static_cast<R>(st.tghost[k - gbase]);
    }
    bool reflected = false;
    bool moved = false;
    int ncross = 0, hits = 0;
    for (;;) {
      R best = static_cast<R>(INFINITY);
      int kb = -1;
#pragma unroll
      for (int kk = 0; kk < NV; ++kk) {
        const R un = DIM == 2 ? u0 * Fx[kk] + u1 * Fy[kk] : u0 * Fx[kk];
        if (un > R(0)) {
          const R xn = DIM == 2 ? Fx[kk] * x + Fy[kk] * y : Fx[kk] * x;
          R te = (Fz[kk] - xn) / un;
          if (te < R(0)) te = R(0);
          if (te < best) {
            best = te;
            kb = kk;
          }
        }
      }
      if (kb < 0 || !(best < t)) {
        x = x + u0 * t;
        if (DIM == 2) y = y + u1 * t;
        break;
      }
      if (++ncross > p.max_cross) {
        // the step fails: later kernels of the step (and of the batch) skip
        atomicOr(st.flags, kFlagRunaway);
        atomicOr(st.halt, 1);
        break;
      }
      x = x + u0 * best;
      if (DIM == 2) y = y + u1 * best;
      R fnx = Fx[0], fny = Fy[0];
      int nb = nbr[0];
#pragma unroll
      for (int kk = 1; kk < NV; ++kk)
        if (kb == kk) {
          fnx = Fx[kk];
          fny = Fy[kk];
          nb = nbr[kk];
        }
      if (nb >= 0) {
        moved = true;
        const int64_t l = static_cast<int64_t>(cell) * NV + kb;
        load_cell(nb);
        if constexpr (F32) {
          // remaining time scales in FP32, the mass with the FP64 ratio;
          // the position moves to the neighbour's anchor
          t = (t - best) * g.lfn32[l].w;
          m = m * g.lfn[l].w;
          const float2 d = g.lda[l];
          x = x + d.x;
          if (DIM == 2) y = y + d.y;
        } else {
          const double r = g.lfn[l].w;
          t = (t - best) * r;
          m = m * r;
        }
        cell = nb;
        continue;
      }
      const int bf = -nb - 1;
      const int ty = g.btype[bf];
      t = t - best;
      if (ty == kBcFarfield || ty == kBcOutflow) {
        exited = true;
        break;
      }
      reflected = true;
      if (ty == kBcSymmetry) {
        if (DIM == 2) {
          const R un = u0 * fnx + u1 * fny;
          const R n0 = u0 - R(2) * un * fnx, n1 = u1 - R(2) * un * fny;
          u0 = n0;
          u1 = n1;
        } else {
          u0 = -u0;
        }
        load_cell(cell);
        continue;
      }
      const double Tw = g.bdata[8 * bf];
      const double sw = sqrt(p.R * Tw);
      double e0, e1, e2, e3, z0, z1;
      rng2(seed, pid, step, kWall, static_cast<uint32_t>(2 * hits), e0, e1);
      rng2(seed, pid, step, kWall, static_cast<uint32_t>(2 * hits + 1), e2, e3);
      ++hits;
      if ((FEAT & kFeatMaxwell) != 0 && ty == kBcMaxwell && !(e3 < g.bdata[8 * bf + 1])) {
        // specular part of a Maxwell wall; the impulse goes to the wall
        const double b0 = u0, b1 = u1;
        if (DIM == 2) {
          const R un = u0 * fnx + u1 * fny;
          const R n0 = u0 - R(2) * un * fnx, n1 = u1 - R(2) * un * fny;
          u0 = n0;
          u1 = n1;
        } else {
          u0 = -u0;
        }
        const double c0 = u0, c1 = u1;
        wall_impulse(p, st, bf, m * (b0 - c0), m * (b1 - c1), 0.0);
        load_cell(cell);
        continue;
      }
      const double vn = sqrt(-2.0 * p.R * Tw * log(e0));
      box_muller(e1, e2, z0, z1);
      const double b0 = u0, b1 = u1, b2 = u2;
      const double fx = fnx, fy = fny;
      double a0, a1, a2;
      if (DIM == 2) {
        const double vt = sw * z0;
        a0 = -vn * fx - vt * fy;
        a1 = -vn * fy + vt * fx;
        a2 = sw * z1;
      } else {
        a0 = -vn * fx;
        a1 = sw * z0;
        a2 = sw * z1;
      }
      // the impulse uses the velocities as stored (rounded in FP32)
      u0 = static_cast<R>(a0);
      u1 = static_cast<R>(a1);
      u2 = static_cast<R>(a2);
      const double c0 = u0, c1 = u1, c2 = u2;
      const double eb = 0.5 * (b0 * b0 + b1 * b1 + b2 * b2);
      const double ea = 0.5 * (c0 * c0 + c1 * c1 + c2 * c2);
      if constexpr ((FEAT & kFeatEi) != 0) {
        // internal energy from the wall temperature (draws of this hit)
        const double eib = ei;
        ei = static_cast<R>((p.R * Tw) *
                            internal_eta(seed, pid, step,
                                         kWallInternalCall0 + static_cast<uint32_t>((hits - 1) * ((p.D + 1) / 2)),
                                         p.D));
        const double eia = ei;
        wall_impulse(p, st, bf, m * (b0 - c0), m * (b1 - c1), m * ((eb + eib) - (ea + eia)));
      } else {
        wall_impulse(p, st, bf, m * (b0 - c0), m * (b1 - c1), m * (eb - ea));
      }
      load_cell(cell);
    }
    // results go to the work store: the committed store stays as it was
    // until the step is complete
    tw.x[k] = x;
    if (DIM == 2) tw.y[k] = y;
    if (reflected) {
      tw.ux[k] = u0;
      tw.uy[k] = u1;
      tw.uz[k] = u2;
      if constexpr ((FEAT & kFeatEi) != 0) tw.ei[k] = ei;
    }
    if (moved) tw.m[k] = m;
    tw.cell[k] = exited ? -1
                        : (cell | (collide ? kCodeCollided : 0) | (reflected ? kCodeReflected : 0) |
                           (moved ? kCodeMoved : 0));
  }
  const bool inside = active && !exited;
  // histogram of the particles ending inside per destination: kept ones in
  // bin `cell`, collided ones (Eq. (51): they end their flight here, enter
  // W^{p,+} of Eq. (30) and are then dropped) in bin nc + cell; one atomic
  // per group, no return value needed
  {
    const int key = inside ? (collide ? static_cast<int>(g.nc) + cell : cell) : -1;
    int leader;
    const uint64_t grp = wave_group(key, leader);
    if (key >= 0 && lane_id() == leader) atomicAdd(&st.count[key], __popcll(grp));
  }
  // step statistics
  const uint64_t me = __ballot(active && exited), mr = __ballot(inside && collide);
  if (lane_id() == 0) {
    int64_t *slot = st.stats + (blockIdx.x % kStatSlots) * kStatN;
    if (me) atomicAdd(reinterpret_cast<unsigned long long *>(&slot[kStatExited]),
                      static_cast<unsigned long long>(__popcll(me)));
    if (mr) atomicAdd(reinterpret_cast<unsigned long long *>(&slot[kStatRemoved]),
                      static_cast<unsigned long long>(__popcll(mr)));
  }
}

// The tracking is bound by the latency of its dependent loads, so occupancy
// pays: the triangle and quad kernels run four wavefronts per SIMD (up to
// 128 VGPRs) without spilling because only a cell's normals, offsets and
// neighbours stay in registers, and not across the reflection code (a face's
// ratio is loaded when it is crossed); polygons with more faces hold more face
// data per lane, and particles with internal energy more state, and get up
// to 256.
template <int DIM, int NV, class R, int FEAT>
__global__ void __launch_bounds__(256, (NV <= 4 && (FEAT & kFeatEi) == 0) ? 4 : 2)
    k_transport(Geo g, Params p, State st, StoreT<R> s, StoreT<R> tw, int64_t cap) {
  if (*st.halt) return;
  const int64_t n_ret = st.roff[g.nc];
  const int64_t gbase = n_ret + st.noff[g.nc];
  const int64_t nt = gbase + *st.nghost;
  const int64_t n_total = nt < cap ? nt : cap;
  const int64_t step = *st.dstep;
  // the grid covers the store capacity, which bounds every step's set
  const int64_t base = blockIdx.x * static_cast<int64_t>(blockDim.x);
  if (base >= n_total) return;  // block-uniform: whole wavefronts take part in the grouping
  transport_one<DIM, NV, R, FEAT>(g, p, st, s, tw, n_ret, gbase, n_total, step, base + threadIdx.x);
}

// Re-sort (counting sort, scatter pass) into the next committed store b:
// cursor[c] starts at the exclusive scan of the counts.  A workgroup claims
// contiguous slots for all its particles of one destination with one atomic:
// each wavefront groups its lanes by destination, the group leaders enter
// the destination in a workgroup table in LDS (open addressing over 512
// entries, so every workgroup of up to 512 particles fits) and take their
// group's offset within the workgroup's run, and one thread per destination
// then claims the run.  Longer runs than per-wavefront claims mean fewer
// partly written lines and fewer global atomics (512-thread workgroups beat
// 256 by 3 %, 1024 was slower again).  Kept particles go to [off[c], off[c+1]) (the next step's
// retained set, sorted by cell); collided ones to [off[nc+c], off[nc+c+1])
// after all kept ones, with only what the tally reads (mass, velocity,
// internal energy).  Positions and cells come from the transport's work
// store tw, velocities and masses from tw where the transport changed them
// (the slot's outcome code says which), else from a.  The order within a
// destination is left open (the tallies are exact sums).
template <int DIM, class R>
__global__ void __launch_bounds__(512) k_scatter(State st, StoreT<R> a, StoreT<R> tw, StoreT<R> b, int64_t cap) {
  constexpr int kSlots = 512;
  __shared__ int skey[kSlots];
  __shared__ int scnt[kSlots];
  __shared__ unsigned long long sbase[kSlots];
  if (*st.halt) return;
  const int64_t ncs = st.nc_scatter;
  const int64_t nt = st.roff[ncs] + st.noff[ncs] + *st.nghost;
  const int64_t n_total = nt < cap ? nt : cap;
  const int64_t base = blockIdx.x * static_cast<int64_t>(blockDim.x);
  if (base >= n_total) return;  // block-uniform
  for (int t = threadIdx.x; t < kSlots; t += blockDim.x) {
    skey[t] = -1;
    scnt[t] = 0;
  }
  __syncthreads();
  const int64_t k = base + threadIdx.x;
  const int code = k < n_total ? tw.cell[k] : -1;
  const bool live = code >= 0;
  const int cell = live ? (code & kCodeCell) : 0;
  const bool col = live && (code & kCodeCollided) != 0;
  const int c = live ? (col ? static_cast<int>(ncs) + cell : cell) : -1;
  int leader;
  const uint64_t grp = wave_group(c, leader);
  int slot = 0, off = 0;
  if (live && lane_id() == leader) {
    slot = static_cast<int>((static_cast<uint32_t>(c) * 2654435761u) >> 23);  // 9 bits: kSlots
    for (;;) {
      const int old = atomicCAS(&skey[slot], -1, c);
      if (old == -1 || old == c) break;
      slot = (slot + 1) & (kSlots - 1);
    }
    off = atomicAdd(&scnt[slot], __popcll(grp));
  }
  const int src = leader >= 0 ? leader : lane_id();
  slot = __shfl(slot, src, 64);
  off = __shfl(off, src, 64);
  __syncthreads();
  for (int t = threadIdx.x; t < kSlots; t += blockDim.x) {
    const int key = skey[t];
    if (key >= 0)
      sbase[t] = atomicAdd(reinterpret_cast<unsigned long long *>(&st.cursor[key]),
                           static_cast<unsigned long long>(scnt[t]));
  }
  __syncthreads();
  if (!live) return;
  const int64_t d = static_cast<int64_t>(sbase[slot]) + off + popc_below(grp);
  const StoreT<R> &uv = (code & kCodeReflected) ? tw : a;
  const StoreT<R> &um = (code & kCodeMoved) ? tw : a;
  // the sources are read once: non-temporal loads (the scatter 302 -> 283 us
  // on the 200x150 cylinder; the tally that follows lost 10 of them)
  b.ux[d] = __builtin_nontemporal_load(&uv.ux[k]);
  b.uy[d] = __builtin_nontemporal_load(&uv.uy[k]);
  b.uz[d] = __builtin_nontemporal_load(&uv.uz[k]);
  if (a.ei) b.ei[d] = __builtin_nontemporal_load(&uv.ei[k]);
  b.m[d] = __builtin_nontemporal_load(&um.m[k]);
  if (col) return;
  b.x[d] = __builtin_nontemporal_load(&tw.x[k]);
  if (DIM == 2) b.y[d] = __builtin_nontemporal_load(&tw.y[k]);
  b.pid[d] = __builtin_nontemporal_load(&a.pid[k]);
  b.cell[d] = cell;
}

// Per-cell tally after the re-sort, one wavefront per cell over its kept
// range [off[c], off[c+1]) and collided range [off[nc+c], off[nc+c+1]):
//   S[c]  = round(sum over kept of m_k Psi_k): the next step's W^p Omega
//           (Eq. (24)); X[c] its exact chunks (normalized);
//   Sp[c] = round(sum over kept and collided): W^{p,+} Omega (Eq. (30));
//   with Pr != 1 the raw moments sum m u_a (|u|^2 + 2 e_i) and
//   sum m u_a u_b that give the heat flux of Eq. (5) once the next step's
//   U is known.
// Every sum is exact (fixed-point chunks, see XWin), so it does not depend on
// the order of the particles within a cell, which the scatter's atomics
// leave open.  Also used at restart (empty collided ranges, Sp = null).

// Adds the exact chunks of one particle's m Psi (RAW false) or raw moments
// (RAW true) to xc.
template <int DIM, bool RAW>
__device__ __forceinline__ void tally_one(const Params &p, double m, double u0, double u1, double u2, double ei,
                                          double (&xc)[32], bool &ok) {
  constexpr int NW = DIM + 2, NLT = kTallyLimbs;
  const double q2 = u0 * u0 + u1 * u1 + u2 * u2;
  if constexpr (!RAW) {
    double t[NW];
    t[0] = m;
    t[1] = m * u0;
    if (DIM == 2) t[2] = m * u1;
    t[NW - 1] = m * (0.5 * q2 + ei);
#pragma unroll
    for (int q = 0; q < NW; ++q) {
      double ch[NLT];
      ok = xs_split<NLT>(t[q], p.xw, ch) && ok;
#pragma unroll
      for (int j = 0; j < NLT; ++j) xc[NLT * q + j] += ch[j];
    }
  } else {
    const double q2i = q2 + 2.0 * ei;
    const double r[5] = {m * u0 * q2i, m * u1 * q2i, m * u0 * u0, m * u0 * u1, m * u1 * u1};
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      double ch[NLT];
      ok = xs_split<NLT>(r[q], p.xm, ch) && ok;
#pragma unroll
      for (int j = 0; j < NLT; ++j) xc[NLT * q + j] += ch[j];
    }
  }
}

// Adds the exact chunks of the particles in [a, b) to xc: of m Psi (RAW
// false) or of the raw moments of the heat flux (RAW true), kTallyLimbs
// chunks per quantity (value kTallyLimbs q + j = chunk j of quantity q).
// Two particles per lane and iteration for m Psi, both loaded before either
// is split (a missing second one has m = 0 and adds zero chunks); one for
// the raw moments, whose five quantities leave no registers for a second.
template <int DIM, bool RAW, class R>
__device__ __forceinline__ void tally_range(const Params &p, const StoreT<R> &s, int64_t a, int64_t b,
                                            double (&xc)[32], bool &ok) {
  if constexpr (RAW) {
    for (int64_t k = a + lane_id(); k < b; k += 64) {
      const double ei = s.ei ? static_cast<double>(s.ei[k]) : 0.0;
      tally_one<DIM, RAW>(p, s.m[k], s.ux[k], s.uy[k], s.uz[k], ei, xc, ok);
    }
    return;
  }
  for (int64_t k = a + lane_id(); k < b; k += 128) {
    const int64_t k2 = k + 64;
    const bool two = k2 < b;
    const double m = s.m[k], u0 = s.ux[k], u1 = s.uy[k], u2 = s.uz[k];
    const double ei = s.ei ? static_cast<double>(s.ei[k]) : 0.0;
    double m2 = 0.0, v0 = 0.0, v1 = 0.0, v2 = 0.0, ej = 0.0;
    if (two) {
      m2 = s.m[k2];
      v0 = s.ux[k2];
      v1 = s.uy[k2];
      v2 = s.uz[k2];
      if (s.ei) ej = s.ei[k2];
    }
    tally_one<DIM, RAW>(p, m, u0, u1, u2, ei, xc, ok);
    tally_one<DIM, RAW>(p, m2, v0, v1, v2, ej, xc, ok);
  }
}

// Chunk totals of one tally pass over [a, b): on return, lane 2 NLT q holds
// the NLT chunk totals of quantity q in L.
template <int DIM, bool RAW, class R>
__device__ __forceinline__ void tally_pass(const Params &p, const StoreT<R> &s, int64_t a, int64_t b,
                                           double (&L)[kTallyLimbs], bool &ok) {
  double xc[32];
#pragma unroll
  for (int v = 0; v < 32; ++v) xc[v] = 0.0;
  tally_range<DIM, RAW>(p, s, a, b, xc, ok);
  // lane l holds the total of value l >> 1
  const double t = wave_sum_spread<32>(xc);
  const int lane = lane_id();
#pragma unroll
  for (int j = 0; j < kTallyLimbs; ++j) L[j] = __shfl(t, (lane + 2 * j) & 63, 64);
}

template <int DIM, bool RAW, class R>
__device__ __forceinline__ void cell_tally(const Geo &g, const Params &p, const StoreT<R> &s, const int64_t *off,
                                           double *S, double *X, double *Sp, double *M, int *flags, int *halt,
                                           int64_t c) {
  constexpr int NW = DIM + 2, NLT = kTallyLimbs;
  const int lane = lane_id();
  const int64_t a = off[c], b = off[c + 1], ca = off[g.nc + c], cb = off[g.nc + c + 1];
  bool ok = (b - a) + (cb - ca) <= (int64_t{1} << 20);
  const int v = lane >> 1, q = v / NLT;
  const bool writer = (lane & 1) == 0 && v % NLT == 0;
  if constexpr (RAW) {
    // raw moments of the kept particles (first, while nothing else is live)
    double Lr[NLT];
    tally_pass<DIM, true>(p, s, a, b, Lr, ok);
    if (writer && q < 5) M[c * 5 + q] = xs_round<NLT>(Lr, p.xm);
  }
  // kept particles: the next step's W^p Omega
  double L[NLT];
  tally_pass<DIM, false>(p, s, a, b, L, ok);
  if (writer && q < NW) {
    S[c * NW + q] = xs_round<NLT>(L, p.xw);
    double Ln[NLT];
#pragma unroll
    for (int j = 0; j < NLT; ++j) Ln[j] = L[j];
    xs_normalize<NLT>(Ln);
#pragma unroll
    for (int j = 0; j < NLT; ++j) X[(c * NW + q) * NLT + j] = Ln[j];
  }
  if (Sp) {
    // collided particles: W^{p,+} Omega is the exact sum over both sets
    double C[NLT];
    tally_pass<DIM, false>(p, s, ca, cb, C, ok);
#pragma unroll
    for (int j = 0; j < NLT; ++j) C[j] += L[j];
    if (writer && q < NW) Sp[c * NW + q] = xs_round<NLT>(C, p.xw);
  }
  if (__ballot(!ok) && lane == 0) {
    atomicOr(flags, kFlagRange);
    atomicOr(halt, 1);
  }
}

// RAW: also the raw moments (Pr != 1).
template <int DIM, class R, bool RAW>
__global__ void __launch_bounds__(256, 4) k_cell_tally(Geo g, Params p, StoreT<R> s, const int64_t *__restrict__ off,
                                                    double *__restrict__ S, double *__restrict__ X,
                                                    double *__restrict__ Sp,
                                                    double *__restrict__ M, int *__restrict__ flags,
                                                    int *__restrict__ halt) {
  const int64_t c = (blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x) >> 6;
  if (c >= g.nc || *halt) return;  // whole wavefront
  cell_tally<DIM, RAW>(g, p, s, off, S, X, Sp, M, flags, halt, c);
}

// ---------------------------------------------------------------------------
// a8: time-averaged wave fluxes, one thread per face (Eqs. (49)-(50)),
// stored as F_j s_j along the face normal (outward of the face's L cell).
// ---------------------------------------------------------------------------
template <int DIM>
__global__ void __launch_bounds__(256, 3) k_face_flux(Geo g, Params p, State st) {
  constexpr int NW = DIM + 2;
  const int64_t fi = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (fi >= g.nf || *st.halt) return;
  const int K = p.K;
  const int L = g.fL[fi], R = g.fR[fi];
  const double2 n = g.fn[fi];
  const double4 xi = g.fxi[fi];  // LL, L, R, RR centroid coordinates along n
  double F[4];
  double wL[4], hL[4];
  to_frame<DIM>(st.W + static_cast<int64_t>(L) * NW, n.x, n.y, wL);
  to_frame<DIM>(st.Wh + static_cast<int64_t>(L) * NW, n.x, n.y, hL);
  const bool hvL = st.hvalid[L] != 0;
  if (R >= 0) {
    const int LL = g.fLL[fi], RR = g.fRR[fi];
    double wR[4], hR[4], wLL[4] = {0, 0, 0, 0}, hLL[4] = {0, 0, 0, 0}, wRR[4] = {0, 0, 0, 0}, hRR[4] = {0, 0, 0, 0};
    to_frame<DIM>(st.W + static_cast<int64_t>(R) * NW, n.x, n.y, wR);
    to_frame<DIM>(st.Wh + static_cast<int64_t>(R) * NW, n.x, n.y, hR);
    const bool hvR = st.hvalid[R] != 0;
    if (LL >= 0) {
      to_frame<DIM>(st.W + static_cast<int64_t>(LL) * NW, n.x, n.y, wLL);
      to_frame<DIM>(st.Wh + static_cast<int64_t>(LL) * NW, n.x, n.y, hLL);
    }
    if (RR >= 0) {
      to_frame<DIM>(st.W + static_cast<int64_t>(RR) * NW, n.x, n.y, wRR);
      to_frame<DIM>(st.Wh + static_cast<int64_t>(RR) * NW, n.x, n.y, hRR);
    }
    double WLf[4], WRf[4], sl[4], sr[4], dW0[4];
    reconstruct(LL >= 0, wLL, xi.x, wL, xi.y, wR, xi.z, WLf, sl);
    reconstruct(RR >= 0, wRR, xi.w, wR, xi.z, wL, xi.y, WRf, sr);
#pragma unroll
    for (int q = 0; q < 4; ++q) dW0[q] = (wR[q] - wL[q]) / (xi.z - xi.y);
    double HLf[4] = {0, 0, 0, 0}, HRf[4] = {0, 0, 0, 0}, shl[4] = {0, 0, 0, 0}, shr[4] = {0, 0, 0, 0};
    if (hvL) {
      const bool okf = LL >= 0 && st.hvalid[LL] != 0 && hvR;
      reconstruct(okf, hLL, xi.x, hL, xi.y, hR, xi.z, HLf, shl);
    }
    if (hvR) {
      const bool okf = RR >= 0 && st.hvalid[RR] != 0 && hvL;
      reconstruct(okf, hRR, xi.w, hR, xi.z, hL, xi.y, HRf, shr);
    }
    flux_interior(WLf, WRf, dW0, hvL, HLf, hvR, HRf, shl, shr, st.dt[L], st.tau[L], st.dt[R], st.tau[R], K, p.Pr,
                  p.wave_only, F);
  } else {
    const int b = -R - 1;
    const int ty = g.btype[b];
    if (ty == kBcWall) {
      flux_wall(wL, hvL, hL, st.dt[L], st.tau[L], g.bdata[8 * b], p.R, K, p.wave_only, F);
    } else {
      double wG[4], hG[4], dW0[4];
      const double z[4] = {0, 0, 0, 0};
      to_frame<DIM>(st.gW + static_cast<int64_t>(b) * NW, n.x, n.y, wG);
      to_frame<DIM>(st.gWh + static_cast<int64_t>(b) * NW, n.x, n.y, hG);
#pragma unroll
      for (int q = 0; q < 4; ++q) dW0[q] = (wG[q] - wL[q]) / (-2.0 * xi.y);
      flux_interior(wL, wG, dW0, hvL, hL, st.ghvalid[b] != 0, hG, z, z, st.dt[L], st.tau[L],
                    st.dt[L], st.gtau[b], K, p.Pr, p.wave_only, F);
      if (ty == kBcMaxwell) {
        // alpha times the diffuse wall's flux plus (1 - alpha) times the
        // mirror-state (specular) flux
        double Fd[4];
        flux_wall(wL, hvL, hL, st.dt[L], st.tau[L], g.bdata[8 * b], p.R, K, p.wave_only, Fd);
        const double a = g.bdata[8 * b + 1];
#pragma unroll
        for (int q = 0; q < 4; ++q) F[q] = a * Fd[q] + (1.0 - a) * F[q];
      }
    }
  }
  double Fl[4];
  from_frame<DIM>(F, n.x, n.y, Fl);
  const double sj = g.fs[fi];
#pragma unroll
  for (int q = 0; q < NW; ++q) st.Fs[fi * NW + q] = Fl[q] * sj;
}

// ---------------------------------------------------------------------------
// a9: W^{n+1} = W^n - dt_i/Omega_i sum_j (+/-) F_j s_j + W^{fr,p}, Eq. (53),
// with W^{fr,p} = W^{p,+} - W^{p,-} (Eq. (29)); faces in fixed local order.
// Invalid results (a cell emptied into vacuum) take the content of the
// particles that ended in the cell, or a vacuum floor state.
// Also the residual sums (exact chunks, per case) and the running mean of
// the density.
// Workgroups from `ublocks` on compute the wall quantities (surface_one)
// instead: one launch for both.
template <int DIM>
__device__ __forceinline__ void surface_one(const Geo &g, const Params &p, const State &st, int64_t w);

template <int DIM>
__global__ void __launch_bounds__(256) k_update(Geo g, Params p, State st, int64_t ublocks) {
  constexpr int NW = DIM + 2;
  if (*st.halt) return;
  if (blockIdx.x >= ublocks) {  // whole workgroups
    surface_one<DIM>(g, p, st, (blockIdx.x - ublocks) * static_cast<int64_t>(blockDim.x) + threadIdx.x);
    return;
  }
  const int64_t step = *st.dstep;
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  double r[2] = {0.0, 0.0};
  bool guarded = false;
  if (i < g.nc) {
    double acc[NW];
#pragma unroll
    for (int q = 0; q < NW; ++q) acc[q] = 0.0;
    for (int k = 0; k < g.NV; ++k) {
      const int64_t l = i * g.NV + k;
      const int fs = g.lface[l];
      if (fs == kNoFace) continue;
      const int f = fs >= 0 ? fs : ~fs;
      const double sg = fs >= 0 ? 1.0 : -1.0;
#pragma unroll
      for (int q = 0; q < NW; ++q) acc[q] += sg * st.Fs[static_cast<int64_t>(f) * NW + q];
    }
    const double vol = g.vol[i];
    const double coef = st.dt[i] / vol;
    double Wn[NW];
#pragma unroll
    for (int q = 0; q < NW; ++q) {
      const double frp = st.Sp[i * NW + q] / vol - st.Sm[i * NW + q] / vol;
      Wn[q] = (st.W[i * NW + q] - coef * acc[q]) + frp;
    }
    const Prim<DIM> s = prim<DIM>(Wn, p.NR);
    if (!prim_ok(s)) {
      guarded = true;
      bool ok = false;
      if (st.Sp[i * NW] > 0.0) {
#pragma unroll
        for (int q = 0; q < NW; ++q) Wn[q] = st.Sp[i * NW + q] / vol;
        ok = prim_ok(prim<DIM>(Wn, p.NR));
      }
      if (!ok) {
        const int cs = case_of(g, i);
        const double rf = 1e-12 * case_val(g, cs, kCaseRho, p.rho_inf);
#pragma unroll
        for (int q = 0; q < NW; ++q) Wn[q] = 0.0;
        Wn[0] = rf;
        Wn[NW - 1] = 0.5 * p.Nd * rf * p.R * case_val(g, cs, kCaseT, p.T_inf);
      }
    }
#pragma unroll
    for (int q = 0; q < NW; ++q) st.W[i * NW + q] = Wn[q];
    const double rho = Wn[0];
    const double d = rho - st.rho_prev[i];
    r[0] = vol * d * d;
    const double sum = st.rho_sum[i] + rho;
    st.rho_sum[i] = sum;
    const double mean = sum / static_cast<double>(step + 1);
    const double dm = step == 0 ? 0.0 : mean - st.rho_mean_prev[i];
    r[1] = vol * dm * dm;
    st.rho_mean_prev[i] = mean;
    st.rho_prev[i] = rho;
  }
  const int lane = lane_id();
  const uint64_t gm = __ballot(guarded);
  if (lane == 0 && gm)
    atomicAdd(reinterpret_cast<unsigned long long *>(&st.stats[(blockIdx.x % kStatSlots) * kStatN + kStatGuard]),
              static_cast<unsigned long long>(__popcll(gm)));
  double rc[2][4];
  bool ok = true;
#pragma unroll
  for (int q = 0; q < 2; ++q) ok = xs_split<4>(r[q], p.xr, rc[q]) && ok;
  if (__ballot(!ok) && lane == 0) atomicOr(st.flags, kFlagResidRange);
  // the sums go to the case of each cell (the cells of a case are
  // contiguous, so a wavefront holds one or two cases)
  const int key = i < g.nc ? case_of(g, i) : -1;
  uint64_t todo = __ballot(key >= 0);
  while (todo) {
    const int l = __ffsll(static_cast<long long>(todo)) - 1;
    const int cs = __builtin_amdgcn_readlane(key, l);
    const bool in = key == cs;
    double v[8];
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int j = 0; j < 4; ++j) v[4 * q + j] = in ? rc[q][j] : 0.0;
    // lane 8 w holds the total of chunk value w = 4 q + j
    const double tot = wave_sum_spread<8>(v);
    if ((lane & 7) == 0 && tot != 0.0) atomicAdd(&st.resid[8 * cs + (lane >> 3)], tot);
    todo &= ~__ballot(in);
  }
}

// a10: wall pressure, shear and heat flux (wave + particle impulses per unit
// area and time), their running sum and EMA (2/1001), and the drag force of
// each wall face w (summed per case in a fixed order by k_finish).  Run by
// extra workgroups of k_update (it needs only the face fluxes, the wall
// impulses and dt).
template <int DIM>
__device__ __forceinline__ void surface_one(const Geo &g, const Params &p, const State &st, int64_t w) {
  constexpr int NW = DIM + 2;
  if (w >= g.nwall) return;
  const int64_t step = *st.dstep;
  const int b = g.wall_b[w];
  const int i = g.bcell[b];
  const int64_t l = static_cast<int64_t>(i) * g.NV + g.bk[b];
  const double4 fl = g.lfn[l];
  const int fs = g.lface[l];
  const int f = fs >= 0 ? fs : ~fs;
  const double s = g.lfs[l];
  double Fl[NW];
#pragma unroll
  for (int q = 0; q < NW; ++q) Fl[q] = st.Fs[static_cast<int64_t>(f) * NW + q] / s;
  double imp[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) imp[q] = xs_round<kTallyLimbs>(st.wimp + (3 * b + q) * kTallyLimbs, p.xw);
  const double nx = fl.x, ny = DIM == 2 ? fl.y : 0.0;
  const double mx = Fl[1], my = DIM == 2 ? Fl[2] : 0.0, eF = Fl[DIM + 1];
  const double sdt = s * st.dt[i];
  const double px = mx + imp[0] / sdt, py = my + (DIM == 2 ? imp[1] / sdt : 0.0);
  double v[3];
  v[0] = px * nx + py * ny;
  v[1] = py * nx - px * ny;
  v[2] = eF + imp[2] / sdt;
  const int cs = case_of(g, i);
  const double ex = case_val(g, cs, kCaseEx, p.u_inf_x / p.U_inf), ey = case_val(g, cs, kCaseEy, p.u_inf_y / p.U_inf);
  st.fd[w] = (px * ex + py * ey) * s;
  constexpr double a = 2.0 / 1001.0;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    st.wlast[3 * w + q] = v[q];
    st.wsum[3 * w + q] += v[q];
    st.wema[3 * w + q] = step == 0 ? v[q] : a * v[q] + (1.0 - a) * st.wema[3 * w + q];
  }
}

// Bookkeeping after a step: per case (one thread each) the residuals from
// their exact chunks and the case's area, C_d from the wall faces' drag
// summed in wall order (last, sum, EMA); then the step's particle counts
// (the statistics slots summed), and the step counter advances (the step is
// committed).  Meeting the residual target (every case's r_avg, r_inst in
// wave-only runs, below it) halts later steps.
__global__ void k_finish(Geo g, Params p, State st, int64_t nc) {
  __shared__ int all_below;
  __shared__ int64_t stat_sum[kStatN];
  if (blockIdx.x != 0 || *st.halt) return;
  const int64_t step = *st.dstep;
  const double tgt = st.scal[kScalTarget];
  if (threadIdx.x == 0) all_below = 1;
  if (threadIdx.x < kStatN) stat_sum[threadIdx.x] = 0;
  __syncthreads();
  // The drag of a case sums its wall faces' terms in wall order.  For each
  // group of blockDim.x cases the block stages the group's terms in LDS,
  // a chunk at a time with every load in flight together, and each case's
  // thread adds its range in order from LDS (the same additions in the same
  // order as one thread walking the array).
  constexpr int kChunk = 2048;
  __shared__ double sfd[kChunk];
  for (int cs0 = 0; cs0 < g.ncase; cs0 += static_cast<int>(blockDim.x)) {
    const int cs = cs0 + static_cast<int>(threadIdx.x);
    const bool has = cs < g.ncase;
    const int cl = (cs0 + static_cast<int>(blockDim.x) < g.ncase ? cs0 + static_cast<int>(blockDim.x) : g.ncase);
    const int64_t gw0 = g.case_wall ? g.case_wall[cs0] : 0, gw1 = g.case_wall ? g.case_wall[cl] : g.nwall;
    const int64_t w0 = has && g.case_wall ? g.case_wall[cs] : 0;
    const int64_t w1 = has ? (g.case_wall ? g.case_wall[cs + 1] : g.nwall) : 0;
    double fsum = 0.0;
    for (int64_t c0 = gw0; c0 < gw1; c0 += kChunk) {
      const int64_t c1 = c0 + kChunk < gw1 ? c0 + kChunk : gw1;
      for (int64_t w = c0 + threadIdx.x; w < c1; w += blockDim.x) sfd[w - c0] = st.fd[w];
      __syncthreads();
      const int64_t a0 = w0 > c0 ? w0 : c0, a1 = w1 < c1 ? w1 : c1;
      // 32 values read ahead of their in-order additions
      int64_t w = a0;
      for (; w + 32 <= a1; w += 32) {
        double v[32];
#pragma unroll
        for (int j = 0; j < 32; ++j) v[j] = sfd[w - c0 + j];
#pragma unroll
        for (int j = 0; j < 32; ++j) fsum += v[j];
      }
      for (; w < a1; ++w) fsum += sfd[w - c0];
      __syncthreads();
    }
    if (!has) continue;
    double *sc = st.scal + cs * kScalN;
    const double rho_inf = case_val(g, cs, kCaseRho, p.rho_inf);
    const double U = case_val(g, cs, kCaseU, p.U_inf), L = case_val(g, cs, kCaseL, p.L_ref);
    const double *rs = st.resid + 8 * cs;
    const double area = st.area[cs];
    sc[kScalRinst] = sqrt(xs_round<4>(rs, p.xr) / area) / rho_inf;
    sc[kScalRavg] = sqrt(xs_round<4>(rs + 4, p.xr) / area) / rho_inf;
    const double cd = fsum / (0.5 * rho_inf * U * U * L);
    constexpr double a = 2.0 / 1001.0;
    sc[kScalCdLast] = cd;
    sc[kScalCdSum] += cd;
    sc[kScalCdEma] = step == 0 ? cd : a * cd + (1.0 - a) * sc[kScalCdEma];
    // particle runs test the running mean's residual (the particle noise
    // floors the instantaneous one); wave-only runs have no noise
    if (!((p.wave_only ? sc[kScalRinst] : sc[kScalRavg]) < tgt)) atomicAnd(&all_below, 0);
  }
  {
    // blockDim.x is a multiple of kStatN: a thread's slots hold one statistic
    int64_t loc = 0;
#pragma unroll 4
    for (int k = threadIdx.x; k < kStatSlots * kStatN; k += blockDim.x) loc += st.stats[k];
    if (loc) atomicAdd(reinterpret_cast<unsigned long long *>(&stat_sum[threadIdx.x % kStatN]),
                       static_cast<unsigned long long>(loc));
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  const int64_t nnew = st.noff[nc] + *st.nghost;
  const int64_t ntot = st.roff[nc] + nnew;
  st.info[kInfoTotal] = ntot;
  st.info[kInfoNew] = nnew;
  st.info[kInfoSumTotal] += ntot;
  st.info[kInfoRemoved] = stat_sum[kStatRemoved];
  st.info[kInfoExited] = stat_sum[kStatExited];
  st.info[kInfoGuard] = stat_sum[kStatGuard];
  st.info[kInfoCapped] = stat_sum[kStatCapped];
  *st.dstep = step + 1;
  // convergence test: the first step n >= 100 with the residual below the target
  if (tgt > 0.0 && step + 1 >= 100 && all_below) {
    *st.flags |= kFlagConverged;
    *st.halt = 1;
  }
}

// Area of each case: the exact sum of its cell volumes (one wavefront per case).
__global__ void k_case_area(Geo g, double *__restrict__ area, XWin w) {
  const int cs = (blockIdx.x * static_cast<int>(blockDim.x) + static_cast<int>(threadIdx.x)) >> 6;
  if (cs >= g.ncase) return;
  const int64_t c0 = g.ccase ? g.case_cell[cs] : 0, c1 = g.ccase ? g.case_cell[cs + 1] : g.nc;
  double xc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t i = c0 + lane_id(); i < c1; i += 64) {
    double ch[4];
    xs_split<4>(g.vol[i], w, ch);
#pragma unroll
    for (int j = 0; j < 4; ++j) xc[j] += ch[j];
  }
  const double tot = wave_sum_spread<4>(xc);
  double L[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) L[j] = __shfl(tot, 16 * j, 64);
  if (lane_id() == 0) area[cs] = xs_round<4>(L, w);
}

// After the count scan, before anything of the step is modified: halt if a
// cell state was invalid, a cell asked for more than 2^20 particles, the
// pre-transport set would not fit the store, or the particle-parallel launches
// (sized on the host from earlier counts) would not cover it.  The bounds are
// recorded so the host can grow the store or the grids and redo this step.
__global__ void k_check(Geo g, State st, int64_t cap, int64_t cover, int64_t cover_new) {
  if (threadIdx.x != 0 || blockIdx.x != 0 || *st.halt) return;
  const int64_t need = st.roff[g.nc] + st.noff[g.nc + g.nb];
  const int64_t nnew = st.noff[g.nc];
  st.info[kInfoNeed] = need;
  st.info[kInfoNeedNew] = nnew;
  if (need > cap) *st.flags |= kFlagCapacity;
  if (need > cover || nnew > cover_new) *st.flags |= kFlagGrid;
  if (*st.flags) *st.halt = 1;
}

// Clears the per-step accumulators of a step (a kernel, not a memset, so
// that the sequence can be captured in a graph).  Does nothing after a halt:
// the steps skipped after a halt must leave the last committed step's
// results as they are.
__global__ void k_zero_many(ZeroList L, const int *__restrict__ halt) {
  if (*halt) return;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  const int64_t i0 = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  for (int b = 0; b < L.count; ++b) {
    uint32_t *p = L.p[b];
    for (int64_t i = i0; i < L.n[b]; i += stride) p[i] = 0u;
  }
}

// Streaming copy of n 16-byte elements: the attainable HBM rate that the
// step's kernels are compared with.  Each thread moves four elements per
// iteration (all four loads issued before the stores).
__global__ void __launch_bounds__(256) k_stream_copy(uint4 *__restrict__ dst, const uint4 *__restrict__ src,
                                                     int64_t n) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    const uint4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
    dst[i] = a;
    dst[i + stride] = b;
    dst[i + 2 * stride] = c;
    dst[i + 3 * stride] = d;
  }
  for (; i < n; i += stride) dst[i] = src[i];
}

// ---------------------------------------------------------------------------
// explicit instantiations
// ---------------------------------------------------------------------------
#define UGK_INST(D)                                                                                       \
  template __global__ void k_init_dt<D>(Geo, Params, const double *, double *, int *);                  \
  template __global__ void k_cell_prep<D>(Geo, Params, State);                                           \
  template __global__ void k_ghost_prep<D>(Geo, Params, State);                                          \
  template __global__ void k_face_flux<D>(Geo, Params, State);                                           \
  template __global__ void k_update<D>(Geo, Params, State, int64_t);
UGK_INST(1)
UGK_INST(2)
#define UGK_INST_P(D, R)                                                                                  \
  template __global__ void k_sample_draw<D, R>(Geo, Params, State, StoreT<R>, int64_t);                  \
  template __global__ void k_sample_match<D, R>(Geo, Params, State, StoreT<R>, int64_t);                 \
  template __global__ void k_sample_shakhov<D, R>(Geo, Params, State, StoreT<R>, int64_t, uint32_t);     \
  template __global__ void k_sample_ghosts<D, R>(Geo, Params, State, StoreT<R>, int64_t);                \
  template __global__ void k_scatter<D, R>(State, StoreT<R>, StoreT<R>, StoreT<R>, int64_t);             \
  template __global__ void k_cell_tally<D, R, false>(Geo, Params, StoreT<R>, const int64_t *, double *,     \
                                                     double *, double *, double *, int *, int *);          \
  template __global__ void k_cell_tally<D, R, true>(Geo, Params, StoreT<R>, const int64_t *, double *,      \
                                                    double *, double *, double *, int *, int *);
UGK_INST_P(1, double)
UGK_INST_P(2, double)
UGK_INST_P(1, float)
UGK_INST_P(2, float)
#define UGK_INST_T(D, N, R, F) \
  template __global__ void k_transport<D, N, R, F>(Geo, Params, State, StoreT<R>, StoreT<R>, int64_t);
#define UGK_INST_TF(D, N, R) UGK_INST_T(D, N, R, 0) UGK_INST_T(D, N, R, 1) UGK_INST_T(D, N, R, 2) UGK_INST_T(D, N, R, 3)
UGK_INST_TF(1, 2, double)
UGK_INST_TF(1, 2, float)
UGK_INST_TF(2, 3, double)
UGK_INST_TF(2, 4, double)
UGK_INST_TF(2, 5, double)
UGK_INST_TF(2, 6, double)
UGK_INST_TF(2, 7, double)
UGK_INST_TF(2, 8, double)
UGK_INST_TF(2, 3, float)
UGK_INST_TF(2, 4, float)
UGK_INST_TF(2, 5, float)
UGK_INST_TF(2, 6, float)
UGK_INST_TF(2, 7, float)
UGK_INST_TF(2, 8, float)

}  // namespace ugk
