// Device data layout and kernel declarations of the UGKWP-LTS library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_math.h"

namespace ugk {

constexpr int kPad = INT32_MIN;      // padding local face (cells with fewer faces)
constexpr int kNoFace = INT32_MIN;   // lface entry of a padding local face
constexpr int kScanBlock = 1024;
constexpr int kMaxCross = 10000;
constexpr int kTallyLimbs = 6;  // chunks of the exact particle tallies (a 192-bit window)

// kBcMaxwell: wall with accommodation alpha (data T_w, alpha), Sec. V.B
enum : int { kBcFarfield = 1, kBcOutflow = 2, kBcWall = 3, kBcSymmetry = 4, kBcMaxwell = 6 };
// kFlagConverged is not an error: the step that reached the residual target
// (scal[kScalTarget] > 0) is done and later steps are skipped
// kFlagRange: a particle term fell outside its exact-summation window (see
// XWin); the step halts before anything is committed
// kFlagResidRange: a residual term fell outside its window; the fields are
// already updated, so the step is committed and the call stops after it
enum : int {
  kFlagInvalid = 1, kFlagRunaway = 2, kFlagOverflow = 4, kFlagCapacity = 8, kFlagGrid = 16, kFlagConverged = 32,
  kFlagRange = 64, kFlagResidRange = 128
};
// kStatCapped: new particles whose Shakhov acceptance-rejection ran out of attempts
enum : int { kStatExited = 0, kStatRemoved = 1, kStatGuard = 2, kStatCapped = 3, kStatN = 4 };
// Step statistics are spread over kStatSlots copies (slot = block id mod
// kStatSlots) so that the per-wave counter updates do not serialize on one
// address; readers sum the slots.
constexpr int kStatSlots = 256;
// Shakhov acceptance-rejection table of a cell: the proposal Maxwellian of
// W^h (U^h, sigma = sqrt(R T^h)), the 6 sigma cutoff, R T, the bound B and
// the target's U, p and heat flux q.
enum : int { kArUhx = 0, kArUhy, kArSig, kArCmax, kArRT, kArBnd, kArUx, kArUy, kArP, kArQx, kArQy, kArN };
// Per-case values: viscosity at T_ref and the freestream reference
// (density, temperature, speed, flow direction, length) of the coefficients.
enum : int { kCaseMu = 0, kCaseRho, kCaseT, kCaseU, kCaseEx, kCaseEy, kCaseL, kCaseN };
enum : int { kScalRinst = 0, kScalRavg, kScalCdLast, kScalCdSum, kScalCdEma, kScalTarget, kScalN };

// Mesh tables (device pointers).  Local faces are padded to NV per cell:
// local face l = cell * NV + k.
struct Geo {
  int NV;
  int64_t nc, nf, nb, nwall;
  const double4 *lfn;    // [nc*NV] outward unit normal (x, y), offset c = n . v_k (z),
                         //   crossing ratio dt_neighbour / dt_cell (w; 1 at boundaries)
  const double *lfs;     // [nc*NV] face length s
  const int *lnb;        // [nc*NV] neighbour cell, -(b+1) for boundary face b, kPad for padding
  const int *lface;      // [nc*NV] global face id f (cell is L) or ~f (cell is R); kNoFace for padding
  const double *vol;     // [nc]
  const double2 *cverts; // [nc*NV] vertex coordinates (1D: x of left/right node)
  const int *nv;         // [nc] vertex count
  const int *fL, *fR;    // [nf] face cells; fR = -(b+1) on the boundary
  const int *fLL, *fRR;  // [nf] cell across the opposite face of L / R (quads, 1D) or -1
  const double2 *fn;     // [nf] unit normal, outward of L
  const double *fs;      // [nf] face length
  const double4 *fxi;    // [nf] centroid coordinates along n from the face midpoint: LL, L, R, RR
  const int *bcell, *bk, *btype; // [nb] interior cell, its local face, BC type
  const double *bdata;   // [nb*8]
  const int *wall_b;     // [nwall] boundary face id of each wall face
  // batches of independent cases (a disjoint union of meshes); ccase is
  // null for a single case, whose parameters are those of Params
  int ncase;
  const int *ccase;           // [nc] case of each cell
  const int64_t *case_cell;   // [ncase + 1] first cell of each case
  const int64_t *case_bface;  // [ncase + 1] first boundary face of each case
  const uint64_t *case_seed;  // [ncase] Philox seed of each case
  const double *case_par;     // [ncase * kCaseN] per-case gas and reference values
  const int64_t *case_wall;   // [ncase + 1] first wall face of each case
  // mixed precision only (particle positions relative to a cell anchor):
  const double2 *anchor; // [nc] anchor of each cell (its centroid)
  const float4 *lfn32;   // [nc*NV] normal (x, y), offset n.(v_k - anchor) (z), crossing ratio (w)
  const float2 *lda;     // [nc*NV] anchor of the cell minus anchor of the neighbour across face k
};

struct Params {
  double R, omega, mu_ref, T_ref, Pr;
  double Nd;   // 3 + D velocity-like degrees of freedom
  double NR;   // Nd * R
  int K;       // lumped degrees of freedom in the face frame, 1 + D
  int D;       // internal degrees of freedom; particles carry |xi|^2 / 2 when D > 0
  double cfl;
  int n_ref;
  int wave_only;  // E = 0: no particles, the waves carry all of g^h
  uint64_t seed;
  double rho_inf, u_inf_x, u_inf_y, U_inf, T_inf, L_ref;
  int max_cross;  // crossings per particle and step before the step fails as a runaway
  // exact-summation windows: particle tallies and wall impulses (xw), raw
  // moments of the heat flux (xm), kTallyLimbs chunks each; residual sums
  // (xr), four chunks
  XWin xw, xm, xr;
};

// Per-step and persistent state (device pointers).
struct State {
  double *W, *Wh, *dt, *tau, *E;
  double2 *tdt;                         // [nc] (tau, dt) for the transport
  int *hvalid;
  double *Sret, *Sretn, *Sm, *Sp;       // tallies sum_k m_k Psi_k [nc*NW]: retained (W^p Omega), W^{p,-}, W^{p,+}
  double *Xret, *Xretn;                 // [nc*NW*kTallyLimbs] the retained tally as normalized exact chunks (window xw)
  double *ar;                           // [nc*kArN] Shakhov acceptance-rejection table (Pr != 1)
  double *Mraw, *Mrawn;                 // [nc*5] sum m u_a |u|^2 (a = x, y), sum m u_x u_x, u_x u_y, u_y u_y
  int64_t *roff;                        // [nc + 1] offsets of the retained (sorted) store
  int *ncount;                          // [nc + nb] new particles per cell / boundary face
  int64_t *noff;                        // [nc + nb + 1] exclusive scan of ncount
  double *mnew;                         // [nc + nb] mass of each new particle
  double *gW, *gWh, *gtau, *gdepth;     // [nb*NW], [nb*NW], [nb], [nb]
  int *ghvalid;                         // [nb]
  int64_t *nghost;                      // entered ghost particles this step
  double *tghost;                       // remaining time of entered ghost particles
  int *count;                           // [2 nc] particles ending in each cell: kept (c), collided (nc + c)
  int64_t *coff;                        // [2 nc + 1] exclusive scan of count
  int64_t *cursor;                      // [2 nc] slot cursor of the scatter
  int64_t nc_scatter;                   // number of cells (for kernels without Geo)
  double *Fs;                           // [nf*NW] time-averaged face flux times s_j
  double *rho_prev, *rho_sum, *rho_mean_prev;
  double *resid;                        // [ncase*2*4] chunks of the residual sums (window xr)
  double *area;                         // [ncase] area of each case (exact sum of the cell volumes)
  double *wimp;                         // [nb*3*kTallyLimbs] chunks of the particle impulse x, y and energy at walls (window xw)
  double *wlast, *wsum, *wema;          // [nwall*3] p, tau, q
  double *fd;                           // [nwall] drag force of each wall face in the step
  double *scal;                         // [ncase*kScalN] per case (the target in case 0's slot)
  int64_t *stats;                       // [kStatSlots * kStatN]
  int *flags;
  int *halt;                            // nonzero: every kernel of later steps returns at once
  int64_t *dstep;                       // step counter (keys the random numbers)
  int64_t *info;                        // [kInfoN] counts of the last committed step and running sums
};
// info: counts of the last committed step (total, new, removed, exited,
// guarded, Shakhov fallbacks), its recorded bounds, and the running work sum
enum : int {
  kInfoTotal = 0, kInfoNew, kInfoNeed, kInfoSumTotal, kInfoNeedNew, kInfoRemoved, kInfoExited, kInfoGuard, kInfoCapped,
  kInfoN
};
// Transport outcome of a slot, held in the work store's cell entry: -1 when
// the particle left the domain; else the cell in the low 28 bits, with bit
// 30 set when it collided (Eq. (51)), bit 29 when a wall or symmetry face
// changed its velocity and bit 28 when it crossed into another cell (its
// mass changed, Eq. (41)); the scatter reads the velocity and the mass from
// the work store only when they changed.  A context holds fewer than 2^28
// cells.
enum : int {
  kCodeCollided = 1 << 30, kCodeReflected = 1 << 29, kCodeMoved = 1 << 28, kCodeCell = (1 << 28) - 1
};

// Particle store, structure of arrays.  R = double: global positions (the
// FP64 path); R = float: positions relative to the cell's anchor and FP32
// velocities (the mixed-precision path).  Masses stay FP64 in both.
template <class R>
struct StoreT {
  R *x, *y, *ux, *uy, *uz;
  R *ei;  // internal energy per unit mass |xi|^2 / 2 (D > 0); nullptr when D = 0
  double *m;
  uint64_t *pid;
  int *cell;
};
using Store = StoreT<double>;
using Store32 = StoreT<float>;

template <int DIM> __global__ void k_init_dt(Geo, Params, const double *, double *, int *);
__global__ void k_init_ratio(Geo, const double *, double4 *);
__global__ void k_init_mixed(Geo, float4 *, float2 *);
template <int DIM> __global__ void k_cell_prep(Geo, Params, State);
template <int DIM> __global__ void k_ghost_prep(Geo, Params, State);
__global__ void k_scan_blocks(const int *, int64_t, int64_t *, int64_t *, const int *);
__global__ void k_scan_add(int64_t *, int64_t, const int64_t *, const int *, int64_t *);
template <int DIM, class R> __global__ void k_sample_draw(Geo, Params, State, StoreT<R>, int64_t);
template <int DIM, class R> __global__ void k_sample_match(Geo, Params, State, StoreT<R>, int64_t);
template <int DIM, class R> __global__ void k_sample_shakhov(Geo, Params, State, StoreT<R>, int64_t, uint32_t);
template <int DIM, class R> __global__ void k_sample_ghosts(Geo, Params, State, StoreT<R>, int64_t);
// Transport specializations: the monatomic, diffuse-wall kernel carries no
// code for the optional features (their registers would cost occupancy).
enum : int { kFeatEi = 1, kFeatMaxwell = 2 };  // particles carry |xi|^2 / 2; Maxwell wall faces exist
template <int DIM, int NV, class R, int FEAT>
__global__ void k_transport(Geo, Params, State, StoreT<R>, StoreT<R>, int64_t);
template <int DIM, class R> __global__ void k_scatter(State, StoreT<R>, StoreT<R>, StoreT<R>, int64_t);
template <int DIM, class R, bool RAW>
__global__ void k_cell_tally(Geo, Params, StoreT<R>, const int64_t *, double *, double *, double *, double *, int *,
                             int *);
__global__ void k_case_area(Geo, double *, XWin);
template <int DIM> __global__ void k_face_flux(Geo, Params, State);
template <int DIM> __global__ void k_update(Geo, Params, State, int64_t);
__global__ void k_finish(Geo, Params, State, int64_t);
__global__ void k_check(Geo, State, int64_t, int64_t, int64_t);
// Up to kZeroMax buffers cleared by one launch (32-bit words each).
constexpr int kZeroMax = 12;
struct ZeroList {
  uint32_t *p[kZeroMax];
  int64_t n[kZeroMax];
  int count;
};
__global__ void k_zero_many(ZeroList, const int *);
__global__ void k_stream_copy(uint4 *, const uint4 *, int64_t);

}  // namespace ugk
