// Host side of the UGKWP-LTS library: mesh tables, device memory, the step
// sequence on one HIP stream, getters and per-kernel event timing.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ugkwp.h"
#include "kernels.h"

using namespace ugk;

// Scratch of ugkwp_step_noalloc: the per-step accumulators of a step (the
// kept/collided histogram and its scatter cursors, the wall-impulse and
// residual chunks, the ghost-entry counter, the step statistics and the
// scan's block sums) in a static device array, for callers that cannot
// allocate.  Every call on a device shares that device's copy; calls that
// overlap on one device race.  Host code uses the address obtained with
// hipGetSymbolAddress, never the array's name.
namespace {
constexpr size_t kNoAllocScratchBytes = size_t{48} << 20;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];


namespace {

enum KernelId {
  kKInitDt, kKCellPrep, kKGhostPrep, kKScan, kKUnused, kKSampleCells, kKSampleGhosts, kKTransport,
  kKFaceFlux, kKUpdate, kKSurface, kKFinish, kKScatter, kKCellTally, kKSampleMatch, kKSampleShakhov, kKCount
};
const char *kKernelNames[kKCount] = {"init_dt",   "cell_prep", "ghost_prep", "scan",      "unused",
                                     "sample_draw", "sample_ghosts", "transport", "face_flux", "update",
                                     "surface",   "finish",    "scatter",   "cell_tally", "sample_match",
                                     "sample_shakhov"};

struct ProfRec {
  int id;
  hipEvent_t a, b;
  double bytes;
};

template <class T>
struct DBuf {
  T *p = nullptr;
  size_t n = 0;
};

}  // namespace

struct ugkwp_ctx {
  int dim = 0, nw = 0, NV = 0;
  int feat = 0;  // transport specialization: kFeatEi (D > 0) | kFeatMaxwell (a Maxwell wall face exists)
  int64_t nc = 0, nf = 0, nb = 0, nwall = 0;
  Params P{};
  int lts = 1;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  // side stream of the face fluxes (they overlap the re-sort) and its fork / join events
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  std::string err;
  // host copies needed by getters
  std::vector<double> h_face_mid;  // [nf*2]
  std::vector<int> h_wall_b, h_bcell, h_bk, h_lface;
  std::vector<double> h_lfn;       // [nc*NV*4]
  // device geometry
  double4 *lfn = nullptr;
  int *lnb = nullptr, *lface = nullptr, *nv = nullptr;
  double *lfs = nullptr, *vol = nullptr;
  double2 *cverts = nullptr;
  int *fL = nullptr, *fR = nullptr, *fLL = nullptr, *fRR = nullptr;
  double2 *fn = nullptr;
  double *fs = nullptr;
  double4 *fxi = nullptr;
  int *bcell = nullptr, *bk = nullptr, *btype = nullptr, *wall_b = nullptr;
  double *bdata = nullptr;
  // state
  State S{};
  int precision = 0;        // 0: FP64 store, 1: mixed (FP32 positions/velocities)
  // particle stores: A the committed set of the current step, B the next
  // committed set (written by the re-sort), T the transport's per-slot
  // results (positions, masses, cells, changed velocities): a step that
  // fails leaves A untouched
  Store A{}, B{}, T{};         // FP64 store (precision 0)
  Store32 A32{}, B32{}, T32{}; // FP32 store (precision 1)
  double2 *anchor = nullptr;
  float4 *lfn32 = nullptr;
  float2 *lda = nullptr;
  std::vector<double> h_anchor;  // [nc*2]
  // cases (one unless built by ugkwp_init_batch)
  int ncase = 1;
  std::vector<int64_t> h_case_cell, h_case_bface;  // [ncase + 1]
  std::vector<double> h_case_par;                  // [ncase * kCaseN]
  int *ccase = nullptr;
  int64_t *case_cell = nullptr, *case_bface = nullptr, *case_wall = nullptr;
  std::vector<int64_t> h_case_wall;                // [ncase + 1] first wall face of each case
  double *Sm_prev = nullptr, *Sp_prev = nullptr;   // W^{p,-}, W^{p,+} (times Omega) of the last committed step
  double *Fs_prev = nullptr;  // F_j s_j of the last committed step (a step writes S.Fs)
  int xw_exp = 0, xm_exp = 0, xr_exp = 0, xa_exp = 0;  // exact-summation window exponents E
  uint64_t *case_seed = nullptr;
  double *case_par = nullptr;
  int64_t cap = 0, n_ret = 0, step = 0;
  int64_t last_total = 0, last_new = 0, last_need = 0, last_need_new = 0;
  int64_t est_total = 0, est_new = 0, est_kept = 0;  // byte-model estimates for the profiler
  int64_t cover = 0, cover_new = 0;  // particles covered by the particle-parallel launches
  int64_t *scan_tmp = nullptr;   // block sums
  int64_t scan_tmp_n = 0;
  int64_t *pinned = nullptr;     // host pinned mailbox
  std::vector<void *> allocs;
  // profiling
  bool prof = false, prof_all = false;
  // tuning
  int32_t batch_steps = 32, use_graph = 1, transport_block = 256, shakhov_lanes = 4, max_crossings = 10000;
  int32_t scatter_block = 512, tally_block = 256, flux_block = 256;
  // ugkwp_step_noalloc: this device's scratch array, and set while such a
  // call runs (no growth, no graph capture, no timing events)
  unsigned char *noalloc_scratch = nullptr;
  bool noalloc = false;
  // captured graph of two steps and the launch arguments it was captured with
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::vector<int64_t> gkey;  // events around every kernel, or the transport only
  std::vector<hipEvent_t> ev_pool;
  std::vector<ProfRec> prof_pending;
  double prof_ms[kKCount] = {0};
  int64_t prof_n[kKCount] = {0};
  double prof_bytes[kKCount] = {0};
  Geo geo() const {
    Geo g;
    g.NV = NV;
    g.nc = nc;
    g.nf = nf;
    g.nb = nb;
    g.nwall = nwall;
    g.lfn = lfn;
    g.lnb = lnb;
    g.lfs = lfs;
    g.lface = lface;
    g.vol = vol;
    g.cverts = cverts;
    g.nv = nv;
    g.fL = fL;
    g.fR = fR;
    g.fLL = fLL;
    g.fRR = fRR;
    g.fn = fn;
    g.fs = fs;
    g.fxi = fxi;
    g.bcell = bcell;
    g.bk = bk;
    g.btype = btype;
    g.bdata = bdata;
    g.wall_b = wall_b;
    g.anchor = anchor;
    g.ncase = ncase;
    g.ccase = ccase;
    g.case_cell = case_cell;
    g.case_bface = case_bface;
    g.case_seed = case_seed;
    g.case_par = case_par;
    g.case_wall = case_wall;
    g.lfn32 = lfn32;
    g.lda = lda;
    return g;
  }
};

namespace {

// Exact-summation window with top exponent E and NL 32-bit chunks.
XWin make_window(int E, int NL) {
  XWin w{};
  w.down = std::ldexp(1.0, 32 - E);
  for (int j = 0; j < NL; ++j) w.up[j] = std::ldexp(1.0, E - 32 * NL + 32 * j);
  return w;
}

int set_err(ugkwp_ctx *c, int code, const char *fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c->err = buf;
  }
  return code;
}

#define HIPCHK(call)                                                                                   \
  do {                                                                                                 \
    hipError_t e_ = (call);                                                                            \
    if (e_ != hipSuccess)                                                                              \
      return set_err(c, e_ == hipErrorOutOfMemory ? UGKWP_ENOMEM : UGKWP_EDEVICE, "%s: %s", #call,      \
                     hipGetErrorString(e_));                                                           \
  } while (0)

template <class T>
int dalloc(ugkwp_ctx *c, T **p, size_t n) {
  void *q = nullptr;
  HIPCHK(hipMalloc(&q, std::max<size_t>(n, 1) * sizeof(T)));
  c->allocs.push_back(q);
  *p = static_cast<T *>(q);
  return UGKWP_OK;
}

void dfree(ugkwp_ctx *c, void *p) {
  if (!p) return;
  auto it = std::find(c->allocs.begin(), c->allocs.end(), p);
  if (it != c->allocs.end()) c->allocs.erase(it);
  (void)hipFree(p);
}

template <class T>
int upload(ugkwp_ctx *c, T **p, const std::vector<T> &h) {
  int rc = dalloc(c, p, h.size());
  if (rc) return rc;
  if (!h.empty()) HIPCHK(hipMemcpyAsync(*p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, c->stream));
  return UGKWP_OK;
}

inline unsigned nblk(int64_t n, int t) { return static_cast<unsigned>(std::max<int64_t>(1, (n + t - 1) / t)); }

// ---------------------------------------------------------------------------
// profiling
// ---------------------------------------------------------------------------
hipEvent_t ev_get(ugkwp_ctx *c) {
  if (!c->ev_pool.empty()) {
    hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
  }
  // timing only: no system-scope fence (that would write back L2 after
  // every timed kernel and slow the step it measures); the times are read
  // after the batch's stream synchronization
  hipEvent_t e;
  if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
  return e;
}

struct ProfScope {
  ugkwp_ctx *c;
  int id;
  double bytes;
  hipEvent_t a = nullptr;
  ProfScope(ugkwp_ctx *c_, int id_, double bytes_) : c(c_), id(id_), bytes(bytes_) {
    if (c->prof && (c->prof_all || id == kKTransport)) {
      a = ev_get(c);
      if (a) (void)hipEventRecord(a, c->stream);
    }
  }
  ~ProfScope() {
    if (c->prof && a) {
      hipEvent_t b = ev_get(c);
      if (b) {
        (void)hipEventRecord(b, c->stream);
        c->prof_pending.push_back({id, a, b, bytes});
      }
    }
  }
};

void prof_harvest(ugkwp_ctx *c) {
  for (auto &r : c->prof_pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      c->prof_ms[r.id] += ms;
      c->prof_n[r.id] += 1;
      c->prof_bytes[r.id] += r.bytes;
    }
    c->ev_pool.push_back(r.a);
    c->ev_pool.push_back(r.b);
  }
  c->prof_pending.clear();
}

// ---------------------------------------------------------------------------
// mesh tables
// ---------------------------------------------------------------------------
struct HostMesh {
  int NV = 0;
  int64_t nc = 0, nf = 0, nb = 0;
  std::vector<double> vol, cen;        // cen [nc*2]
  std::vector<double> lfn;             // [nc*NV*4]
  std::vector<int> lnb, lface, nv;     // [nc*NV], [nc*NV], [nc]
  std::vector<double> cverts;          // [nc*NV*2]
  std::vector<int> fL, fR, fkL, fkR, fLL, fRR;
  std::vector<double> fn, fs, fmid, fxi;
  std::vector<int> bcell, bk;
};

// Geometry by fan triangulation from vertex 0 (area, centroid); CCW edge
// d = v_{k+1} - v_k has outward unit normal (d_y, -d_x)/|d|, length |d| and
// offset n . v_k.  Faces are numbered in order of first appearance over
// (cell, local face); L is that first cell and n its outward normal.
int build_mesh(ugkwp_ctx *c, const ugkwp_mesh *m, HostMesh &h) {
  const int dim = m->dim;
  const int64_t nc = m->n_cells, nb = m->n_bfaces;
  h.nc = nc;
  h.nb = nb;
  if (dim == 1) {
    if (m->n_nodes != nc + 1) return set_err(c, UGKWP_EINVAL, "1D mesh needs n_nodes = n_cells + 1");
    h.NV = 2;
  } else {
    if (!m->cell_ptr || !m->cell_nodes) return set_err(c, UGKWP_EINVAL, "2D mesh needs cell_ptr/cell_nodes");
    int mx = 0;
    for (int64_t i = 0; i < nc; ++i) {
      const int64_t nvv = m->cell_ptr[i + 1] - m->cell_ptr[i];
      if (nvv < 3 || nvv > 8) return set_err(c, UGKWP_EINVAL, "cell %lld has %lld vertices", (long long)i, (long long)nvv);
      mx = std::max<int>(mx, static_cast<int>(nvv));
    }
    h.NV = mx;
  }
  const int NV = h.NV;
  h.vol.assign(nc, 0.0);
  h.cen.assign(nc * 2, 0.0);
  h.lfn.assign(nc * NV * 4, 0.0);
  h.lnb.assign(nc * NV, kPad);
  h.lface.assign(nc * NV, kNoFace);
  h.nv.assign(nc, 0);
  h.cverts.assign(nc * NV * 2, 0.0);
  h.bcell.assign(nb, -1);
  h.bk.assign(nb, -1);
  const double *v = m->nodes;
  if (dim == 1) {
    for (int64_t i = 0; i < nc; ++i) {
      const double xl = v[i], xr = v[i + 1];
      if (!(xr > xl)) return set_err(c, UGKWP_EINVAL, "1D nodes not increasing at %lld", (long long)i);
      h.vol[i] = xr - xl;
      h.cen[2 * i] = 0.5 * (xl + xr);
      h.nv[i] = 2;
      double *f0 = &h.lfn[(i * NV + 0) * 4], *f1 = &h.lfn[(i * NV + 1) * 4];
      f0[0] = -1.0; f0[1] = 0.0; f0[2] = -xl; f0[3] = 1.0;
      f1[0] = 1.0;  f1[1] = 0.0; f1[2] = xr;  f1[3] = 1.0;
      h.lnb[i * NV + 0] = static_cast<int>(i - 1);
      h.lnb[i * NV + 1] = static_cast<int>(i + 1);
      h.cverts[(i * NV + 0) * 2] = xl;
      h.cverts[(i * NV + 1) * 2] = xr;
    }
    int seen0 = 0, seen1 = 0;
    for (int64_t b = 0; b < nb; ++b) {
      const int64_t nd = m->bface_nodes[b];
      if (nd == 0) {
        h.lnb[0] = static_cast<int>(-(b + 1)); h.bcell[b] = 0; h.bk[b] = 0; ++seen0;
      } else if (nd == nc) {
        h.lnb[(nc - 1) * NV + 1] = static_cast<int>(-(b + 1)); h.bcell[b] = static_cast<int>(nc - 1); h.bk[b] = 1; ++seen1;
      } else {
        return set_err(c, UGKWP_EINVAL, "1D boundary face on interior node %lld", (long long)nd);
      }
    }
    if (seen0 != 1 || seen1 != 1) return set_err(c, UGKWP_EINVAL, "1D mesh needs one boundary face at each end");
  } else {
    struct Edge {
      int64_t a, b, cell, k;
    };
    std::vector<Edge> E;
    E.reserve(m->cell_ptr[nc]);
    for (int64_t i = 0; i < nc; ++i) {
      const int64_t s0 = m->cell_ptr[i];
      const int nvv = static_cast<int>(m->cell_ptr[i + 1] - s0);
      const int64_t *id = m->cell_nodes + s0;
      for (int k = 0; k < nvv; ++k)
        if (id[k] < 0 || id[k] >= m->n_nodes) return set_err(c, UGKWP_EINVAL, "cell %lld node out of range", (long long)i);
      h.nv[i] = nvv;
      const double x0 = v[2 * id[0]], y0 = v[2 * id[0] + 1];
      double area = 0.0, cx = 0.0, cy = 0.0;
      for (int t = 0; t + 2 < nvv; ++t) {
        const double xa = v[2 * id[t + 1]], ya = v[2 * id[t + 1] + 1];
        const double xb = v[2 * id[t + 2]], yb = v[2 * id[t + 2] + 1];
        const double At = 0.5 * ((xa - x0) * (yb - y0) - (xb - x0) * (ya - y0));
        area += At;
        cx += At * ((x0 + xa + xb) / 3.0);
        cy += At * ((y0 + ya + yb) / 3.0);
      }
      if (!(area > 0.0)) return set_err(c, UGKWP_EINVAL, "cell %lld has non-positive area (not CCW?)", (long long)i);
      h.vol[i] = area;
      h.cen[2 * i] = cx / area;
      h.cen[2 * i + 1] = cy / area;
      for (int k = 0; k < nvv; ++k) {
        const int64_t a = id[k], b = id[(k + 1) % nvv], bb = id[(k + 2) % nvv];
        const double dx = v[2 * b] - v[2 * a], dy = v[2 * b + 1] - v[2 * a + 1];
        const double ex = v[2 * bb] - v[2 * b], ey = v[2 * bb + 1] - v[2 * b + 1];
        if (!(dx * ey - dy * ex > 0.0)) return set_err(c, UGKWP_EINVAL, "cell %lld is not strictly convex/CCW", (long long)i);
        const double len = std::sqrt(dx * dx + dy * dy);
        const double nx = dy / len, ny = -dx / len;
        double *f = &h.lfn[(i * NV + k) * 4];
        f[0] = nx;
        f[1] = ny;
        f[2] = nx * v[2 * a] + ny * v[2 * a + 1];
        f[3] = len;
        h.cverts[(i * NV + k) * 2] = v[2 * a];
        h.cverts[(i * NV + k) * 2 + 1] = v[2 * a + 1];
        E.push_back({std::min(a, b), std::max(a, b), i, k});
      }
    }
    std::sort(E.begin(), E.end(), [](const Edge &p, const Edge &q) {
      if (p.a != q.a) return p.a < q.a;
      if (p.b != q.b) return p.b < q.b;
      if (p.cell != q.cell) return p.cell < q.cell;
      return p.k < q.k;
    });
    std::vector<Edge> Bv(nb);
    for (int64_t b = 0; b < nb; ++b) {
      const int64_t a = m->bface_nodes[2 * b], d = m->bface_nodes[2 * b + 1];
      Bv[b] = {std::min(a, d), std::max(a, d), b, 0};
    }
    std::sort(Bv.begin(), Bv.end(), [](const Edge &p, const Edge &q) { return p.a != q.a ? p.a < q.a : p.b < q.b; });
    size_t ib = 0;
    for (size_t e = 0; e < E.size();) {
      if (e + 1 < E.size() && E[e + 1].a == E[e].a && E[e + 1].b == E[e].b) {
        if (e + 2 < E.size() && E[e + 2].a == E[e].a && E[e + 2].b == E[e].b)
          return set_err(c, UGKWP_EINVAL, "edge shared by more than two cells");
        h.lnb[E[e].cell * NV + E[e].k] = static_cast<int>(E[e + 1].cell);
        h.lnb[E[e + 1].cell * NV + E[e + 1].k] = static_cast<int>(E[e].cell);
        e += 2;
      } else {
        while (ib < Bv.size() && (Bv[ib].a < E[e].a || (Bv[ib].a == E[e].a && Bv[ib].b < E[e].b))) ++ib;
        if (ib >= Bv.size() || Bv[ib].a != E[e].a || Bv[ib].b != E[e].b)
          return set_err(c, UGKWP_EINVAL, "open edge (%lld,%lld) not in the boundary list", (long long)E[e].a, (long long)E[e].b);
        const int64_t b = Bv[ib].cell;
        h.lnb[E[e].cell * NV + E[e].k] = static_cast<int>(-(b + 1));
        h.bcell[b] = static_cast<int>(E[e].cell);
        h.bk[b] = static_cast<int>(E[e].k);
        ++e;
      }
    }
  }
  for (int64_t b = 0; b < nb; ++b)
    if (h.bcell[b] < 0) return set_err(c, UGKWP_EINVAL, "boundary face %lld matches no cell edge", (long long)b);
  // global faces
  std::vector<int> lf(nc * NV, -1);
  int64_t nf = 0;
  for (int64_t i = 0; i < nc; ++i) {
    for (int k = 0; k < h.nv[i]; ++k) {
      const int64_t l = i * NV + k;
      if (lf[l] >= 0) continue;
      const int f = static_cast<int>(nf++);
      lf[l] = f;
      h.lface[l] = f;
      h.fL.push_back(static_cast<int>(i));
      h.fkL.push_back(k);
      h.fn.push_back(h.lfn[l * 4]);
      h.fn.push_back(h.lfn[l * 4 + 1]);
      h.fs.push_back(h.lfn[l * 4 + 3]);
      if (dim == 1) {
        h.fmid.push_back(k == 0 ? v[i] : v[i + 1]);
        h.fmid.push_back(0.0);
      } else {
        const int kn = (k + 1) % h.nv[i];
        h.fmid.push_back(0.5 * (h.cverts[l * 2] + h.cverts[(i * NV + kn) * 2]));
        h.fmid.push_back(0.5 * (h.cverts[l * 2 + 1] + h.cverts[(i * NV + kn) * 2 + 1]));
      }
      const int nbr = h.lnb[l];
      if (nbr >= 0) {
        int found = -1;
        for (int k2 = 0; k2 < h.nv[nbr]; ++k2)
          if (h.lnb[static_cast<int64_t>(nbr) * NV + k2] == i && lf[static_cast<int64_t>(nbr) * NV + k2] < 0) {
            found = k2;
            break;
          }
        if (found < 0) return set_err(c, UGKWP_EINVAL, "inconsistent neighbour table");
        lf[static_cast<int64_t>(nbr) * NV + found] = f;
        h.lface[static_cast<int64_t>(nbr) * NV + found] = ~f;
        h.fR.push_back(nbr);
        h.fkR.push_back(found);
      } else {
        h.fR.push_back(nbr);
        h.fkR.push_back(-1);
      }
    }
  }
  h.nf = nf;
  // reconstruction stencil: the cell across the opposite face (1D: 1-k; quads: k+2)
  auto opposite = [&](int cell, int k) -> int {
    int ko;
    if (dim == 1) ko = 1 - k;
    else if (h.nv[cell] == 4) ko = (k + 2) % 4;
    else return -1;
    const int nb2 = h.lnb[static_cast<int64_t>(cell) * NV + ko];
    return nb2 >= 0 ? nb2 : -1;
  };
  h.fLL.resize(nf);
  h.fRR.resize(nf);
  h.fxi.assign(nf * 4, 0.0);
  for (int64_t f = 0; f < nf; ++f) {
    const int L = h.fL[f], R = h.fR[f];
    const double nx = h.fn[2 * f], ny = h.fn[2 * f + 1];
    const double mx = h.fmid[2 * f], my = h.fmid[2 * f + 1];
    auto xi = [&](int cell) { return (h.cen[2 * cell] - mx) * nx + (h.cen[2 * cell + 1] - my) * ny; };
    h.fLL[f] = R >= 0 ? opposite(L, h.fkL[f]) : -1;
    h.fRR[f] = R >= 0 ? opposite(R, h.fkR[f]) : -1;
    h.fxi[4 * f + 1] = xi(L);
    if (R >= 0) h.fxi[4 * f + 2] = xi(R);
    if (h.fLL[f] >= 0) h.fxi[4 * f + 0] = xi(h.fLL[f]);
    if (h.fRR[f] >= 0) h.fxi[4 * f + 3] = xi(h.fRR[f]);
  }
  return UGKWP_OK;
}

// ---------------------------------------------------------------------------
// scan helper: out[0..n] = exclusive scan of in[0..n), out[n] = total
// ---------------------------------------------------------------------------
// Block sums of an exclusive scan of up to n values, reserved at init (no
// allocation may happen while a graph is being captured).
int reserve_scan(ugkwp_ctx *c, int64_t n) {
  const int64_t nblocks = std::max<int64_t>(1, (n + kScanBlock) / kScanBlock);
  if (nblocks + 1 <= c->scan_tmp_n) return UGKWP_OK;
  dfree(c, c->scan_tmp);
  c->scan_tmp = nullptr;
  int rc = dalloc(c, &c->scan_tmp, static_cast<size_t>(nblocks + 1));
  if (rc) return rc;
  c->scan_tmp_n = nblocks + 1;
  return UGKWP_OK;
}

int scan(ugkwp_ctx *c, const int *in, int64_t n, int64_t *out, int64_t *copy = nullptr) {
  const int64_t nblocks = std::max<int64_t>(1, (n + kScanBlock) / kScanBlock);
  if (nblocks + 1 > c->scan_tmp_n) return set_err(c, UGKWP_EDEVICE, "scan of %lld values exceeds its reserve", (long long)n);
  ProfScope ps(c, kKScan, 12.0 * static_cast<double>(n));
  hipLaunchKernelGGL(k_scan_blocks, dim3(nblocks), dim3(kScanBlock), 0, c->stream, in, n, out, c->scan_tmp,
                     c->S.halt);
  hipLaunchKernelGGL(k_scan_add, dim3(nblocks), dim3(kScanBlock), 0, c->stream, out, n, c->scan_tmp, c->S.halt,
                     copy);
  HIPCHK(hipGetLastError());
  return UGKWP_OK;
}

template <class R>
int alloc_store(ugkwp_ctx *c, StoreT<R> &s, int64_t n, bool with_pid = true) {
  int rc = 0;
  rc |= dalloc(c, &s.x, n);
  if (c->dim == 2) rc |= dalloc(c, &s.y, n);
  rc |= dalloc(c, &s.ux, n);
  rc |= dalloc(c, &s.uy, n);
  rc |= dalloc(c, &s.uz, n);
  if (c->P.D > 0) rc |= dalloc(c, &s.ei, n);
  rc |= dalloc(c, &s.m, n);
  if (with_pid) rc |= dalloc(c, &s.pid, n);
  rc |= dalloc(c, &s.cell, n);
  return rc ? UGKWP_ENOMEM : UGKWP_OK;
}

template <class R>
void free_store(ugkwp_ctx *c, StoreT<R> &s) {
  dfree(c, s.x);
  dfree(c, s.y);
  dfree(c, s.ux);
  dfree(c, s.uy);
  dfree(c, s.uz);
  dfree(c, s.ei);
  dfree(c, s.m);
  dfree(c, s.pid);
  dfree(c, s.cell);
  s = StoreT<R>{};
}

template <class R>
int copy_store(ugkwp_ctx *c, const StoreT<R> &from, const StoreT<R> &to, int64_t n) {
  if (n <= 0) return UGKWP_OK;
  const size_t d8 = n * sizeof(double), dr = n * sizeof(R);
  HIPCHK(hipMemcpyAsync(to.x, from.x, dr, hipMemcpyDeviceToDevice, c->stream));
  if (c->dim == 2) HIPCHK(hipMemcpyAsync(to.y, from.y, dr, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(to.ux, from.ux, dr, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(to.uy, from.uy, dr, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(to.uz, from.uz, dr, hipMemcpyDeviceToDevice, c->stream));
  if (from.ei) HIPCHK(hipMemcpyAsync(to.ei, from.ei, dr, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(to.m, from.m, d8, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(to.pid, from.pid, n * sizeof(uint64_t), hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(to.cell, from.cell, n * sizeof(int), hipMemcpyDeviceToDevice, c->stream));
  return UGKWP_OK;
}

// Grow the particle buffers to hold at least `need` particles (retained kept).
template <class R>
int grow_stores(ugkwp_ctx *c, StoreT<R> &A, StoreT<R> &B, StoreT<R> &T, int64_t ncap) {
  StoreT<R> A2{}, B2{}, T2{};
  int rc = alloc_store(c, A2, ncap);
  if (!rc) rc = alloc_store(c, B2, ncap);
  if (!rc) rc = alloc_store(c, T2, ncap, false);
  if (rc) return set_err(c, UGKWP_ENOMEM, "cannot grow particle store to %lld", (long long)ncap);
  rc = copy_store(c, A, A2, c->n_ret);
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(c->stream));
  free_store(c, A);
  free_store(c, B);
  free_store(c, T);
  A = A2;
  B = B2;
  T = T2;
  return UGKWP_OK;
}

int ensure_capacity(ugkwp_ctx *c, int64_t need) {
  if (need <= c->cap) return UGKWP_OK;
  const int64_t ncap = std::max<int64_t>(need + need / 4 + 1024, c->cap + c->cap / 2);
  if (ncap > (int64_t{1} << 31) - 256)
    return set_err(c, UGKWP_EOVERFLOW, "particle store of %lld exceeds 2^31", (long long)ncap);
  const int rc = c->precision ? grow_stores(c, c->A32, c->B32, c->T32, ncap) : grow_stores(c, c->A, c->B, c->T, ncap);
  if (rc) return rc;
  dfree(c, c->S.tghost);
  c->S.tghost = nullptr;
  if (dalloc(c, &c->S.tghost, ncap))
    return set_err(c, UGKWP_ENOMEM, "cannot grow particle work arrays");
  c->cap = ncap;
  return UGKWP_OK;
}

void swap_buffers(ugkwp_ctx *c) {
  std::swap(c->A, c->B);
  std::swap(c->A32, c->B32);
  std::swap(c->S.Sret, c->S.Sretn);
  std::swap(c->S.Xret, c->S.Xretn);
  std::swap(c->S.Sm, c->Sm_prev);
  std::swap(c->S.Sp, c->Sp_prev);
  std::swap(c->S.Fs, c->Fs_prev);
  std::swap(c->S.roff, c->S.coff);
  std::swap(c->S.Mraw, c->S.Mrawn);
}

// Collects buffers to clear with one k_zero_many launch.
struct Zeroer {
  ZeroList L{};
  int64_t total = 0;
  void add(void *p, int64_t words) {
    L.p[L.count] = static_cast<uint32_t *>(p);
    L.n[L.count] = words;
    ++L.count;
    total = std::max(total, words);
  }
  void launch(ugkwp_ctx *c) {
    hipLaunchKernelGGL(k_zero_many, dim3(std::min<unsigned>(nblk(total, 256), 1024u)), dim3(256), 0, c->stream, L,
                       c->S.halt);
  }
};

// Enqueues one step on the stream; no host synchronization.  Every launch
// size depends only on host-known constants (mesh sizes, capacity, grid
// estimates); the particle counts live on the device.  The host swaps the
// double-buffered pointers; after a halted batch it restores their parity.
// The transport specialization for the context's features.
template <int DIM, int NV, class R>
void launch_transport(ugkwp_ctx *c, const Geo &g, const State &S, const StoreT<R> &A, const StoreT<R> &T, dim3 gr,
                      dim3 bl) {
  switch (c->feat) {
    case 0: hipLaunchKernelGGL((k_transport<DIM, NV, R, 0>), gr, bl, 0, c->stream, g, c->P, S, A, T, c->cap); break;
    case kFeatEi:
      hipLaunchKernelGGL((k_transport<DIM, NV, R, kFeatEi>), gr, bl, 0, c->stream, g, c->P, S, A, T, c->cap);
      break;
    case kFeatMaxwell:
      hipLaunchKernelGGL((k_transport<DIM, NV, R, kFeatMaxwell>), gr, bl, 0, c->stream, g, c->P, S, A, T, c->cap);
      break;
    default:
      hipLaunchKernelGGL((k_transport<DIM, NV, R, kFeatEi | kFeatMaxwell>), gr, bl, 0, c->stream, g, c->P, S, A, T,
                         c->cap);
      break;
  }
}

// Per-cell tally of the store s over the ranges of `off` (Pr != 1 also the
// raw moments of the heat flux).
template <int DIM, class R>
void launch_tally(ugkwp_ctx *c, const Geo &g, const StoreT<R> &s, const int64_t *off, double *S, double *X,
                  double *Sp, double *M) {
  const dim3 gr(nblk(c->nc * 64, c->tally_block)), bl(c->tally_block);
  if (c->P.Pr != 1.0)
    hipLaunchKernelGGL((k_cell_tally<DIM, R, true>), gr, bl, 0, c->stream, g, c->P, s, off, S, X, Sp, M, c->S.flags,
                       c->S.halt);
  else
    hipLaunchKernelGGL((k_cell_tally<DIM, R, false>), gr, bl, 0, c->stream, g, c->P, s, off, S, X, Sp, M,
                       c->S.flags, c->S.halt);
}

template <int DIM>
void launch_face_flux(ugkwp_ctx *c, const Geo &g, const State &S, hipStream_t st) {
  hipLaunchKernelGGL(k_face_flux<DIM>, dim3(nblk(c->nf, c->flux_block)), dim3(c->flux_block), 0, st, g, c->P, S);
}

template <int DIM, class R>
int enqueue_step(ugkwp_ctx *c, const StoreT<R> &A, const StoreT<R> &B, const StoreT<R> &T) {
  const int NW = DIM + 2;
  const Geo g = c->geo();
  State &S = c->S;
  const int64_t nc = c->nc, nb = c->nb;
  {
    ProfScope ps(c, kKCellPrep, 160.0 * nc);
    hipLaunchKernelGGL(k_cell_prep<DIM>, dim3(nblk(nc, 256)), dim3(256), 0, c->stream, g, c->P, S);
  }
  if (nb > 0) {
    ProfScope ps(c, kKGhostPrep, 200.0 * nb);
    hipLaunchKernelGGL(k_ghost_prep<DIM>, dim3(nblk(nb, 256)), dim3(256), 0, c->stream, g, c->P, S);
  }
  int rc = scan(c, S.ncount, nc + nb, S.noff);
  if (rc) return rc;
  hipLaunchKernelGGL(k_check, dim3(1), dim3(64), 0, c->stream, g, S, c->cap, c->cover, c->cover_new);
  {
    // the step's accumulators, cleared once the step is known to proceed
    // (a halted step leaves the last committed step's values in place)
    Zeroer z;
    z.add(S.count, 2 * nc);
    z.add(S.wimp, std::max<int64_t>(nb, 1) * 3 * kTallyLimbs * 2);
    z.add(S.resid, 8 * 2 * c->ncase);
    z.add(S.nghost, 2);
    z.add(S.stats, kStatSlots * kStatN * 2);
    z.launch(c);
  }
  // bytes of one particle record: positions and velocities, mass, pid, cell
  const double rec = (DIM + 3) * static_cast<double>(sizeof(R)) + 20.0;
  // particle-parallel grids cover c->cover particles (c->cover_new new ones);
  // a step whose counts exceed them halts in k_check and is redone with
  // larger grids.  Blocks past the step's count return at once.
  const unsigned gcap = static_cast<unsigned>(nblk(c->cover, c->scatter_block));
  const unsigned gnew = static_cast<unsigned>(nblk(c->cover_new, 256));
  {
    ProfScope ps(c, kKSampleCells, rec * c->est_new);
    hipLaunchKernelGGL((k_sample_draw<DIM, R>), dim3(gnew), dim3(256), 0, c->stream, g, c->P, S, A, c->cap);
  }
  if (c->P.Pr != 1.0) {
    ProfScope ps(c, kKSampleShakhov, 40.0 * c->est_new);
    // one wavefront per 64 / shakhov_lanes new particles
    const unsigned gsh = nblk((c->cover_new + 64 / c->shakhov_lanes - 1) / (64 / c->shakhov_lanes) * 64, 256);
    hipLaunchKernelGGL((k_sample_shakhov<DIM, R>), dim3(gsh), dim3(256), 0, c->stream, g, c->P, S, A, c->cap,
                       static_cast<uint32_t>(c->shakhov_lanes));
  }
  {
    ProfScope ps(c, kKSampleMatch, 48.0 * c->est_new + (8.0 * 2 * NW + 24.0) * nc);
    hipLaunchKernelGGL((k_sample_match<DIM, R>), dim3(nblk(nc * 16, 256)), dim3(256), 0, c->stream, g, c->P, S, A,
                       c->cap);
  }
  if (nb > 0) {
    ProfScope ps(c, kKSampleGhosts, 0.0);
    hipLaunchKernelGGL((k_sample_ghosts<DIM, R>), dim3(nblk(nb * 64, 256)), dim3(256), 0, c->stream, g, c->P, S, A,
                       c->cap);
  }
  {
    // transport reads a record and writes x, (y), m, cell and the keep flag
    const double wr = DIM * static_cast<double>(sizeof(R)) + 16.0;
    ProfScope ps(c, kKTransport, (rec + wr) * c->est_total);
    const dim3 gr(nblk(c->cover, c->transport_block)), bl(c->transport_block);
    if constexpr (DIM == 1) {
      launch_transport<DIM, 2, R>(c, g, S, A, T, gr, bl);
    } else {
      switch (c->NV) {
        case 3: launch_transport<2, 3, R>(c, g, S, A, T, gr, bl); break;
        case 4: launch_transport<2, 4, R>(c, g, S, A, T, gr, bl); break;
        case 5: launch_transport<2, 5, R>(c, g, S, A, T, gr, bl); break;
        case 6: launch_transport<2, 6, R>(c, g, S, A, T, gr, bl); break;
        case 7: launch_transport<2, 7, R>(c, g, S, A, T, gr, bl); break;
        default: launch_transport<2, 8, R>(c, g, S, A, T, gr, bl); break;
      }
    }
  }
  // The face fluxes need only the cell states of the step's start: they run
  // on the side stream beside the re-sort, which leaves most of the device's
  // registers free (with per-kernel timing on, in order on the library
  // stream instead).
  const bool side = !c->prof;
  if (side) {
    HIPCHK(hipEventRecord(c->ev_fork, c->stream));
    HIPCHK(hipStreamWaitEvent(c->side, c->ev_fork, 0));
    launch_face_flux<DIM>(c, g, S, c->side);
    HIPCHK(hipEventRecord(c->ev_join, c->side));
  }
  // kept particles per cell in count[0, nc), collided ones in count[nc, 2 nc)
  // the scan also sets the scatter's cursors to the offsets
  rc = scan(c, S.count, 2 * nc, S.coff, S.cursor);
  if (rc) return rc;
  {
    ProfScope ps(c, kKScatter, (2.0 * rec + 4.0) * c->est_kept);
    hipLaunchKernelGGL((k_scatter<DIM, R>), dim3(gcap), dim3(c->scatter_block), 0, c->stream, S, A, T, B, c->cap);
  }
  {
    const double rd = 8.0 * NW;  // m and the velocity components of a kept particle
    ProfScope ps(c, kKCellTally, rd * c->est_kept + (16.0 + 8.0 * NW * 6) * nc);
    launch_tally<DIM, R>(c, g, B, S.coff, S.Sretn, S.Xretn, S.Sp, S.Mrawn);
  }
  if (side) {
    HIPCHK(hipStreamWaitEvent(c->stream, c->ev_join, 0));
  } else {
    ProfScope ps(c, kKFaceFlux, 408.0 * c->nf);
    launch_face_flux<DIM>(c, g, S, c->stream);
  }
  {
    // the cells' update, and the wall quantities in workgroups after them
    ProfScope ps(c, kKUpdate, 350.0 * nc + 150.0 * c->nwall);
    const int64_t ub = nblk(nc, 256);
    hipLaunchKernelGGL(k_update<DIM>, dim3(static_cast<unsigned>(ub + nblk(c->nwall, 256))), dim3(256), 0, c->stream,
                       g, c->P, S, ub);
  }
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(std::max(256, std::min(1024, (c->ncase + 63) / 64 * 64))), 0,
                     c->stream, g, c->P, S, nc);
  HIPCHK(hipGetLastError());
  swap_buffers(c);
  return UGKWP_OK;
}

int enqueue(ugkwp_ctx *c) {
  if (c->precision)
    return c->dim == 1 ? enqueue_step<1, float>(c, c->A32, c->B32, c->T32)
                       : enqueue_step<2, float>(c, c->A32, c->B32, c->T32);
  return c->dim == 1 ? enqueue_step<1, double>(c, c->A, c->B, c->T) : enqueue_step<2, double>(c, c->A, c->B, c->T);
}

int check_flags(ugkwp_ctx *c) {
  int flags = 0;
  HIPCHK(hipMemcpyAsync(&flags, c->S.flags, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  if (flags) {
    // the error is reported here; later steps start clean
    HIPCHK(hipMemsetAsync(c->S.flags, 0, sizeof(int), c->stream));
    HIPCHK(hipMemsetAsync(c->S.halt, 0, sizeof(int), c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
  }
  if (flags & kFlagInvalid) return set_err(c, UGKWP_ENUMERIC, "invalid cell state");
  if (flags & kFlagRunaway) return set_err(c, UGKWP_ENUMERIC, "runaway particle tracking");
  if (flags & kFlagOverflow) return set_err(c, UGKWP_EOVERFLOW, "more than 2^20 particles in one cell");
  if (flags & kFlagRange) return set_err(c, UGKWP_ENUMERIC, "a tally term outside its exact-summation window");
  return UGKWP_OK;
}

// Reads the retained count and the last step's counts (host sync).
int sync_counts(ugkwp_ctx *c) {
  int64_t info[kInfoN];
  HIPCHK(hipMemcpyAsync(&c->pinned[4], c->S.roff + c->nc, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipMemcpyAsync(info, c->S.info, sizeof info, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  c->n_ret = c->pinned[4];
  c->last_total = info[kInfoTotal];
  c->last_new = info[kInfoNew];
  c->last_need = info[kInfoNeed];
  c->last_need_new = info[kInfoNeedNew];
  return UGKWP_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

}  // extern "C"

namespace {

bool params_ok(const ugkwp_params *par) {
  return par->R > 0 && par->mu_ref > 0 && par->T_ref > 0 && par->Pr > 0 && par->cfl > 0 && par->n_ref > 0 &&
         par->D >= 0 && par->D <= 64 && par->rho_inf > 0 && par->T_inf > 0 && par->L_ref > 0 &&
         (par->dt_source == 0 || par->dt_source == 1);
}

// The state Eq. (33) reads for a case: its initial field W0 (dt_source 0), or
// its freestream reference state repeated over its n cells (dt_source 1), so
// that a start from another field keeps the freestream start's time steps.
void dt_field(const ugkwp_params *q, int dim, int64_t n, const double *W0, std::vector<double> &out) {
  const int nw = dim + 2;
  if (n <= 0) return;
  if (q->dt_source == 0) {
    out.insert(out.end(), W0, W0 + n * nw);
    return;
  }
  const double rho = q->rho_inf, ux = q->u_inf_x, uy = dim == 2 ? q->u_inf_y : 0.0;
  const double E = rho * (0.5 * (ux * ux + uy * uy) + 0.5 * (3 + q->D) * q->R * q->T_inf);
  for (int64_t i = 0; i < n; ++i) {
    out.push_back(rho);
    out.push_back(rho * ux);
    if (dim == 2) out.push_back(rho * uy);
    out.push_back(E);
  }
}

// Per-case table row of a parameter set.
void case_row(const ugkwp_params *q, double *row) {
  const double U = std::sqrt(q->u_inf_x * q->u_inf_x + q->u_inf_y * q->u_inf_y);
  row[kCaseMu] = q->mu_ref;
  row[kCaseRho] = q->rho_inf;
  row[kCaseT] = q->T_inf;
  row[kCaseU] = U;
  row[kCaseEx] = q->u_inf_x / U;
  row[kCaseEy] = q->u_inf_y / U;
  row[kCaseL] = q->L_ref;
}

// Builds a context for `mesh` (for a batch, the disjoint union of the cases'
// meshes) with the shared parameters of `par` and, for a batch, the cases'
// cell and boundary-face ranges, seeds and per-case table.
int init_impl(ugkwp_ctx *c, const ugkwp_mesh *mesh, const ugkwp_params *par, const double *W0, const double *Wdt,
              int ncase, const std::vector<int64_t> &case_cell, const std::vector<int64_t> &case_bface,
              const std::vector<uint64_t> &seeds, const std::vector<double> &case_par) {
  if (mesh->dim != 1 && mesh->dim != 2) return set_err(c, UGKWP_EINVAL, "dim must be 1 or 2");
  if (mesh->n_cells <= 0 || mesh->n_cells >= (int64_t{1} << 31) - 1 - mesh->n_bfaces)
    return set_err(c, UGKWP_EINVAL, "n_cells + n_bfaces must be in [1, 2^31)");
  if (mesh->n_cells > kCodeCell) return set_err(c, UGKWP_EINVAL, "a context holds fewer than 2^28 cells");
  for (int k = 0; k < ncase; ++k)
    if ((case_cell[k + 1] - case_cell[k]) + (case_bface[k + 1] - case_bface[k]) >= (1 << 24) - 1)
      return set_err(c, UGKWP_EINVAL, "n_cells + n_bfaces of a case must be below 2^24");
  if (!params_ok(par)) return set_err(c, UGKWP_EINVAL, "invalid parameters");
  c->ncase = ncase;
  c->h_case_cell = case_cell;
  c->h_case_bface = case_bface;
  c->h_case_par = case_par;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return set_err(c, UGKWP_EDEVICE, "no HIP device");
  c->dim = mesh->dim;
  c->nw = mesh->dim + 2;
  c->lts = par->lts;
  if (par->precision != 0 && par->precision != 1) return set_err(c, UGKWP_EINVAL, "precision must be 0 or 1");
  c->precision = par->precision;
  Params &P = c->P;
  P.R = par->R;
  P.omega = par->omega;
  P.mu_ref = par->mu_ref;
  P.T_ref = par->T_ref;
  P.Pr = par->Pr;
  P.Nd = static_cast<double>(3 + par->D);
  P.NR = P.Nd * par->R;
  P.K = 1 + par->D;
  P.D = par->D;
  P.cfl = par->cfl;
  P.n_ref = par->n_ref;
  P.wave_only = par->wave_only ? 1 : 0;
  P.seed = par->seed;
  P.rho_inf = par->rho_inf;
  P.u_inf_x = par->u_inf_x;
  P.u_inf_y = par->u_inf_y;
  P.U_inf = std::sqrt(par->u_inf_x * par->u_inf_x + par->u_inf_y * par->u_inf_y);
  P.T_inf = par->T_inf;
  P.L_ref = par->L_ref;
  if (!(P.U_inf > 0)) return set_err(c, UGKWP_EINVAL, "u_inf must be nonzero");
  if (par->stream) {
    c->stream = static_cast<hipStream_t>(par->stream);
  } else {
    HIPCHK(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
    c->own_stream = true;
  }
  HIPCHK(hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
  HIPCHK(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
  for (int64_t b = 0; b < mesh->n_bfaces; ++b)
    if ((mesh->bface_type[b] < 1 || mesh->bface_type[b] > 4) && mesh->bface_type[b] != UGKWP_BC_WALL_MAXWELL)
      return set_err(c, UGKWP_EINVAL, "boundary face %lld has unknown type", (long long)b);
  HostMesh h;
  int rc = build_mesh(c, mesh, h);
  if (rc) return rc;
  c->NV = h.NV;
  c->nc = h.nc;
  c->nf = h.nf;
  c->nb = h.nb;
  const int64_t nc = c->nc, nb = c->nb, nw = c->nw;
  c->h_face_mid = h.fmid;
  c->h_bcell = h.bcell;
  c->h_bk = h.bk;
  c->h_lfn = h.lfn;
  c->h_anchor = h.cen;
  c->h_lface = h.lface;
  std::vector<int> wall_b, btype(mesh->bface_type, mesh->bface_type + nb);
  c->feat = c->P.D > 0 ? kFeatEi : 0;
  for (int64_t b = 0; b < nb; ++b) {
    if (btype[b] == UGKWP_BC_WALL_DIFFUSE || btype[b] == UGKWP_BC_WALL_MAXWELL) wall_b.push_back(static_cast<int>(b));
    if (btype[b] == UGKWP_BC_WALL_MAXWELL) c->feat |= kFeatMaxwell;
  }
  c->h_wall_b = wall_b;
  c->nwall = static_cast<int64_t>(wall_b.size());
  // device geometry
  // face record: normal, offset and (set on the device from the time steps)
  // the crossing ratio; lengths separately
  std::vector<double4> lfn4(nc * c->NV);
  std::vector<double> lfs(nc * c->NV);
  for (int64_t l = 0; l < nc * c->NV; ++l) {
    lfn4[l] = make_double4(h.lfn[4 * l], h.lfn[4 * l + 1], h.lfn[4 * l + 2], 1.0);
    lfs[l] = h.lfn[4 * l + 3];
  }
  std::vector<double2> cv2(nc * c->NV), fn2(c->nf);
  for (int64_t l = 0; l < nc * c->NV; ++l) cv2[l] = make_double2(h.cverts[2 * l], h.cverts[2 * l + 1]);
  for (int64_t f = 0; f < c->nf; ++f) fn2[f] = make_double2(h.fn[2 * f], h.fn[2 * f + 1]);
  std::vector<double4> fxi4(c->nf);
  for (int64_t f = 0; f < c->nf; ++f) fxi4[f] = make_double4(h.fxi[4 * f], h.fxi[4 * f + 1], h.fxi[4 * f + 2], h.fxi[4 * f + 3]);
  std::vector<double> bdata(mesh->bface_data, mesh->bface_data + nb * 8);
  if (ncase > 1) {
    std::vector<int> cc(nc);
    for (int k = 0; k < ncase; ++k)
      for (int64_t i = case_cell[k]; i < case_cell[k + 1]; ++i) cc[i] = k;
    if ((rc = upload(c, &c->ccase, cc)) || (rc = upload(c, &c->case_cell, case_cell)) ||
        (rc = upload(c, &c->case_bface, case_bface)) || (rc = upload(c, &c->case_seed, seeds)) ||
        (rc = upload(c, &c->case_par, case_par)))
      return rc;
  }
  if ((rc = upload(c, &c->lfn, lfn4)) || (rc = upload(c, &c->lfs, lfs)) || (rc = upload(c, &c->lnb, h.lnb)) || (rc = upload(c, &c->lface, h.lface)) ||
      (rc = upload(c, &c->nv, h.nv)) || (rc = upload(c, &c->vol, h.vol)) || (rc = upload(c, &c->cverts, cv2)) ||
      (rc = upload(c, &c->fL, h.fL)) || (rc = upload(c, &c->fR, h.fR)) || (rc = upload(c, &c->fLL, h.fLL)) ||
      (rc = upload(c, &c->fRR, h.fRR)) || (rc = upload(c, &c->fn, fn2)) || (rc = upload(c, &c->fs, h.fs)) ||
      (rc = upload(c, &c->fxi, fxi4)) || (rc = upload(c, &c->bcell, h.bcell)) || (rc = upload(c, &c->bk, h.bk)) ||
      (rc = upload(c, &c->btype, btype)) || (rc = upload(c, &c->bdata, bdata)) || (rc = upload(c, &c->wall_b, wall_b)))
    return rc;
  // state
  State &S = c->S;
  std::vector<double> W(W0, W0 + nc * nw);
  if ((rc = upload(c, &S.W, W))) return rc;
  const size_t ncw = nc * nw, nbw = std::max<int64_t>(nb, 1) * nw;
  const size_t nb1 = std::max<int64_t>(nb, 1), nwl1 = std::max<int64_t>(c->nwall, 1);
  if (dalloc(c, &S.Wh, ncw) || dalloc(c, &S.dt, nc) || dalloc(c, &S.tau, nc) || dalloc(c, &S.tdt, nc) ||
      dalloc(c, &S.E, nc) || dalloc(c, &S.hvalid, nc) || dalloc(c, &S.Sret, ncw) || dalloc(c, &S.Sretn, ncw) ||
      dalloc(c, &S.Sm, ncw) || dalloc(c, &S.Sp, ncw) || dalloc(c, &c->Sm_prev, ncw) || dalloc(c, &c->Sp_prev, ncw) ||
      dalloc(c, &S.Xret, ncw * kTallyLimbs) || dalloc(c, &S.Xretn, ncw * kTallyLimbs) ||
      dalloc(c, &S.roff, 2 * nc + 1) || dalloc(c, &S.cursor, 2 * nc) || dalloc(c, &S.ar, nc * kArN) ||
      dalloc(c, &S.Mraw, nc * 5) || dalloc(c, &S.Mrawn, nc * 5) || dalloc(c, &S.ncount, nc + nb) ||
      dalloc(c, &S.noff, nc + nb + 1) || dalloc(c, &S.mnew, nc + nb) || dalloc(c, &S.gW, nbw) ||
      dalloc(c, &S.gWh, nbw) || dalloc(c, &S.gtau, nb1) || dalloc(c, &S.gdepth, nb1) ||
      dalloc(c, &S.ghvalid, nb1) || dalloc(c, &S.nghost, 1) || dalloc(c, &S.count, 2 * nc) ||
      dalloc(c, &S.coff, 2 * nc + 1) || dalloc(c, &S.Fs, c->nf * nw) || dalloc(c, &c->Fs_prev, c->nf * nw) || dalloc(c, &S.rho_prev, nc) ||
      dalloc(c, &S.rho_sum, nc) || dalloc(c, &S.rho_mean_prev, nc) || dalloc(c, &S.resid, 8 * ncase) ||
      dalloc(c, &S.area, ncase) || dalloc(c, &S.wimp, nb1 * 3 * kTallyLimbs) || dalloc(c, &S.wlast, nwl1 * 3) ||
      dalloc(c, &S.wsum, nwl1 * 3) || dalloc(c, &S.wema, nwl1 * 3) || dalloc(c, &S.fd, nwl1) ||
      dalloc(c, &S.scal, ncase * kScalN) || dalloc(c, &S.stats, kStatSlots * kStatN) || dalloc(c, &S.flags, 1) ||
      dalloc(c, &S.halt, 1) || dalloc(c, &S.dstep, 1) || dalloc(c, &S.info, kInfoN))
    return set_err(c, UGKWP_ENOMEM, "device allocation failed");
  S.nc_scatter = nc;
  HIPCHK(hipMemsetAsync(S.Sret, 0, ncw * sizeof(double), c->stream));
  HIPCHK(hipMemsetAsync(S.Xret, 0, ncw * kTallyLimbs * sizeof(double), c->stream));
  HIPCHK(hipMemsetAsync(S.Sm, 0, ncw * sizeof(double), c->stream));
  HIPCHK(hipMemsetAsync(S.Sp, 0, ncw * sizeof(double), c->stream));
  HIPCHK(hipMemsetAsync(c->Sm_prev, 0, ncw * sizeof(double), c->stream));
  HIPCHK(hipMemsetAsync(c->Sp_prev, 0, ncw * sizeof(double), c->stream));
  HIPCHK(hipMemsetAsync(S.Fs, 0, c->nf * nw * sizeof(double), c->stream));
  HIPCHK(hipMemsetAsync(c->Fs_prev, 0, c->nf * nw * sizeof(double), c->stream));
  HIPCHK(hipMemsetAsync(S.roff, 0, (2 * nc + 1) * sizeof(int64_t), c->stream));
  HIPCHK(hipMemsetAsync(S.coff, 0, (2 * nc + 1) * sizeof(int64_t), c->stream));
  HIPCHK(hipMemsetAsync(S.ar, 0, nc * kArN * sizeof(double), c->stream));
  HIPCHK(hipMemsetAsync(S.Mraw, 0, nc * 5 * sizeof(double), c->stream));
  HIPCHK(hipMemsetAsync(S.count, 0, 2 * nc * sizeof(int), c->stream));
  HIPCHK(hipMemsetAsync(S.rho_sum, 0, nc * sizeof(double), c->stream));
  HIPCHK(hipMemsetAsync(S.rho_mean_prev, 0, nc * sizeof(double), c->stream));
  HIPCHK(hipMemsetAsync(S.wsum, 0, nwl1 * 3 * sizeof(double), c->stream));
  HIPCHK(hipMemsetAsync(S.wlast, 0, nwl1 * 3 * sizeof(double), c->stream));
  HIPCHK(hipMemsetAsync(S.wema, 0, nwl1 * 3 * sizeof(double), c->stream));
  HIPCHK(hipMemsetAsync(S.wimp, 0, nb1 * 3 * kTallyLimbs * sizeof(double), c->stream));
  HIPCHK(hipMemsetAsync(S.resid, 0, 8 * ncase * sizeof(double), c->stream));
  HIPCHK(hipMemsetAsync(S.scal, 0, ncase * kScalN * sizeof(double), c->stream));
  HIPCHK(hipMemsetAsync(S.stats, 0, kStatSlots * kStatN * sizeof(int64_t), c->stream));
  HIPCHK(hipMemsetAsync(S.flags, 0, sizeof(int), c->stream));
  HIPCHK(hipMemsetAsync(S.halt, 0, sizeof(int), c->stream));
  HIPCHK(hipMemsetAsync(S.dstep, 0, sizeof(int64_t), c->stream));
  HIPCHK(hipMemsetAsync(S.info, 0, kInfoN * sizeof(int64_t), c->stream));
  HIPCHK(hipMemsetAsync(S.nghost, 0, sizeof(int64_t), c->stream));
  // exact-summation windows (see XWin): E from bounds of the initial state,
  // the far-field states and the geometry with generous headroom; a term
  // beyond its window fails the step (ENUMERIC)
  {
    double content = 0.0, vmax = 0.0, rho_max = 0.0, area_max = 0.0;
    const double R = par->R;
    auto visit = [&](const double *Ws, double vol) {
      const double rho = Ws[0];
      double mom = 0.0;
      for (int d = 0; d < c->dim; ++d) mom += Ws[1 + d] * Ws[1 + d];
      mom = std::sqrt(mom);
      const double E = Ws[nw - 1];
      content = std::max(content, vol * (std::fabs(rho) + mom + std::fabs(E)));
      rho_max = std::max(rho_max, std::fabs(rho));
      if (rho > 0) {
        const double U = mom / rho;
        const double e = E - 0.5 * rho * U * U;
        const double T = std::max(0.0, 2.0 * e / ((3.0 + par->D) * R * rho));
        vmax = std::max(vmax, U + 15.0 * std::sqrt(R * T));
      }
    };
    for (int64_t i = 0; i < nc; ++i) visit(W0 + i * nw, h.vol[i]);
    for (int64_t b = 0; b < nb; ++b) {
      const double *d = mesh->bface_data + 8 * b;
      const int64_t i = h.bcell[b];
      if (btype[b] == UGKWP_BC_FARFIELD) {
        double Wg[4] = {d[0], d[0] * d[1], 0.0, 0.0};
        if (c->dim == 2) Wg[2] = d[0] * d[2];
        Wg[nw - 1] = 0.5 * d[0] * (d[1] * d[1] + (c->dim == 2 ? d[2] * d[2] : 0.0)) + 0.5 * (3.0 + par->D) * d[0] * R * d[3];
        visit(Wg, h.vol[i]);
      } else if (btype[b] == UGKWP_BC_WALL_DIFFUSE || btype[b] == UGKWP_BC_WALL_MAXWELL) {
        vmax = std::max(vmax, 15.0 * std::sqrt(R * std::fabs(d[0])));
      }
    }
    for (int k = 0; k < ncase; ++k) {
      double a = 0.0;
      for (int64_t i = case_cell[k]; i < case_cell[k + 1]; ++i) a += h.vol[i];
      area_max = std::max(area_max, a);
    }
    if (!(content > 0.0) || !std::isfinite(content) || !std::isfinite(vmax))
      return set_err(c, UGKWP_ENUMERIC, "invalid initial state");
    auto expo = [](double v) { return static_cast<int>(std::ceil(std::log2(v))); };
    c->xw_exp = expo(content) + 12;
    c->xm_exp = c->xw_exp + expo(2.0 * std::max(vmax, 1.0)) + 2;
    c->xr_exp = expo(area_max * std::max(rho_max, 1e-300) * std::max(rho_max, 1e-300)) + 25;
    c->xa_exp = expo(area_max) + 1;
    P.xw = make_window(c->xw_exp, kTallyLimbs);
    P.xm = make_window(c->xm_exp, kTallyLimbs);
    P.xr = make_window(c->xr_exp, 4);
    P.max_cross = c->max_crossings;
    // walls of each case (wall faces are numbered in boundary-face order)
    c->h_case_wall.assign(ncase + 1, 0);
    for (int k = 0; k < ncase; ++k) {
      int64_t n = 0;
      for (int64_t b = case_bface[k]; b < case_bface[k + 1]; ++b)
        if (btype[b] == UGKWP_BC_WALL_DIFFUSE || btype[b] == UGKWP_BC_WALL_MAXWELL) ++n;
      c->h_case_wall[k + 1] = c->h_case_wall[k] + n;
    }
    if ((rc = upload(c, &c->case_wall, c->h_case_wall))) return rc;
    Geo ga = c->geo();
    hipLaunchKernelGGL(k_case_area, dim3(nblk(ncase * 64, 256)), dim3(256), 0, c->stream, ga, S.area,
                       make_window(c->xa_exp, 4));
    HIPCHK(hipGetLastError());
  }
  // rho_prev = initial density
  {
    std::vector<double> r(nc);
    for (int64_t i = 0; i < nc; ++i) r[i] = W0[i * nw];
    HIPCHK(hipMemcpyAsync(S.rho_prev, r.data(), nc * sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
  }
  if ((rc = reserve_scan(c, std::max(2 * nc, nc + nb)))) return rc;
  {
    // this device's copy of the no-allocation scratch array, once per device
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return set_err(c, UGKWP_EDEVICE, "device id %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
      void *ptr = nullptr;
      const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !ptr)
        return set_err(c, UGKWP_EDEVICE, "scratch array address: %s", hipGetErrorString(e));
      g_scratch_ptr[dev] = ptr;
    }
    c->noalloc_scratch = static_cast<unsigned char *>(g_scratch_ptr[dev]);
  }
  void *pin = nullptr;
  HIPCHK(hipHostMalloc(&pin, 8 * sizeof(int64_t), hipHostMallocDefault));
  c->pinned = static_cast<int64_t *>(pin);
  // a1: local time steps
  const Geo g = c->geo();
  double *Wd = S.W;
  if (Wdt != W0) {
    if ((rc = dalloc(c, &Wd, nc * nw))) return rc;
    HIPCHK(hipMemcpyAsync(Wd, Wdt, nc * nw * sizeof(double), hipMemcpyHostToDevice, c->stream));
  }
  {
    ProfScope ps(c, kKInitDt, 80.0 * nc);
    if (c->dim == 1)
      hipLaunchKernelGGL(k_init_dt<1>, dim3(nblk(nc, 256)), dim3(256), 0, c->stream, g, P, Wd, S.dt, S.flags);
    else
      hipLaunchKernelGGL(k_init_dt<2>, dim3(nblk(nc, 256)), dim3(256), 0, c->stream, g, P, Wd, S.dt, S.flags);
  }
  HIPCHK(hipGetLastError());
  rc = check_flags(c);
  if (Wd != S.W) dfree(c, Wd);
  if (rc) return set_err(c, UGKWP_ENUMERIC, "invalid initial state");
  if (!c->lts) {
    // global time step, Eq. (34): the minimum over each case's cells
    std::vector<double> dt(nc);
    HIPCHK(hipMemcpy(dt.data(), S.dt, nc * sizeof(double), hipMemcpyDeviceToHost));
    for (int k = 0; k < ncase; ++k) {
      const auto a = dt.begin() + case_cell[k], b = dt.begin() + case_cell[k + 1];
      const double m = *std::min_element(a, b);
      std::fill(a, b, m);
    }
    HIPCHK(hipMemcpy(S.dt, dt.data(), nc * sizeof(double), hipMemcpyHostToDevice));
  }
  Geo g2 = c->geo();
  hipLaunchKernelGGL(k_init_ratio, dim3(nblk(nc * c->NV, 256)), dim3(256), 0, c->stream, g2, S.dt, c->lfn);
  HIPCHK(hipGetLastError());
  if (c->precision) {
    // cell anchors (centroids) and the FP32 tracking tables
    std::vector<double2> anc(nc);
    for (int64_t i = 0; i < nc; ++i) anc[i] = make_double2(c->h_anchor[2 * i], c->h_anchor[2 * i + 1]);
    if ((rc = upload(c, &c->anchor, anc))) return rc;
    if (dalloc(c, &c->lfn32, nc * c->NV) || dalloc(c, &c->lda, nc * c->NV))
      return set_err(c, UGKWP_ENOMEM, "device allocation failed");
    Geo g3 = c->geo();
    hipLaunchKernelGGL(k_init_mixed, dim3(nblk(nc * c->NV, 256)), dim3(256), 0, c->stream, g3, c->lfn32, c->lda);
    HIPCHK(hipGetLastError());
  }
  const int64_t cap0 = par->particle_capacity > 0 ? par->particle_capacity
                                                  : std::max<int64_t>(4096, 2 * static_cast<int64_t>(par->n_ref) * nc);
  if ((rc = ensure_capacity(c, cap0))) return rc;
  HIPCHK(hipStreamSynchronize(c->stream));
  return UGKWP_OK;
}

}  // namespace

extern "C" {

int ugkwp_init(const ugkwp_mesh *mesh, const ugkwp_params *par, const double *W0, ugkwp_ctx **out) {
  if (!out) return UGKWP_EINVAL;
  *out = nullptr;
  ugkwp_ctx *c = new (std::nothrow) ugkwp_ctx();
  if (!c) return UGKWP_ENOMEM;
  *out = c;
  if (!mesh || !par || !W0) return set_err(c, UGKWP_EINVAL, "null argument");
  if (!params_ok(par)) return set_err(c, UGKWP_EINVAL, "invalid parameters");
  std::vector<double> row(kCaseN);
  case_row(par, row.data());
  if (mesh->dim != 1 && mesh->dim != 2) return set_err(c, UGKWP_EINVAL, "dim must be 1 or 2");
  std::vector<double> Wdt;
  if (par->dt_source) dt_field(par, mesh->dim, mesh->n_cells, W0, Wdt);
  return init_impl(c, mesh, par, W0, par->dt_source ? Wdt.data() : W0, 1, {0, mesh->n_cells}, {0, mesh->n_bfaces},
                   {par->seed}, row);
}

int ugkwp_init_batch(int32_t n_cases, const ugkwp_mesh *meshes, const ugkwp_params *params,
                     const double *const *W0, ugkwp_ctx **out) {
  if (!out) return UGKWP_EINVAL;
  *out = nullptr;
  ugkwp_ctx *c = new (std::nothrow) ugkwp_ctx();
  if (!c) return UGKWP_ENOMEM;
  *out = c;
  if (n_cases < 1 || !meshes || !params || !W0) return set_err(c, UGKWP_EINVAL, "null argument or no case");
  const ugkwp_params &p0 = params[0];
  const ugkwp_mesh &m0 = meshes[0];
  for (int k = 0; k < n_cases; ++k) {
    const ugkwp_params &q = params[k];
    if (!params_ok(&q) || !W0[k] || meshes[k].dim != m0.dim || meshes[k].n_cells <= 0)
      return set_err(c, UGKWP_EINVAL, "case %d: invalid parameters, mesh or W0", k);
    if (q.R != p0.R || q.omega != p0.omega || q.T_ref != p0.T_ref || q.Pr != p0.Pr || q.D != p0.D ||
        q.cfl != p0.cfl || q.n_ref != p0.n_ref || q.lts != p0.lts || q.precision != p0.precision ||
        q.wave_only != p0.wave_only ||
        q.stream != p0.stream)
      return set_err(c, UGKWP_EINVAL, "case %d: gas, CFL, N_ref, LTS, precision and stream must equal case 0's", k);
  }
  // the disjoint union of the meshes
  const int dim = m0.dim, nw = dim + 2;
  std::vector<double> nodes, bdata, W, Wdt;
  std::vector<int64_t> cell_ptr{0}, cell_nodes, bnodes;
  std::vector<int32_t> btype;
  std::vector<int64_t> case_cell{0}, case_bface{0};
  std::vector<uint64_t> seeds;
  std::vector<double> cpar(static_cast<size_t>(n_cases) * kCaseN);
  int64_t node_off = 0;
  for (int k = 0; k < n_cases; ++k) {
    const ugkwp_mesh &m = meshes[k];
    if (dim == 1) return set_err(c, UGKWP_EINVAL, "batches are 2D");
    nodes.insert(nodes.end(), m.nodes, m.nodes + m.n_nodes * dim);
    for (int64_t i = 0; i < m.n_cells; ++i) cell_ptr.push_back(cell_ptr.back() + (m.cell_ptr[i + 1] - m.cell_ptr[i]));
    for (int64_t q = 0; q < m.cell_ptr[m.n_cells]; ++q) cell_nodes.push_back(m.cell_nodes[q] + node_off);
    for (int64_t q = 0; q < m.n_bfaces * dim; ++q) bnodes.push_back(m.bface_nodes[q] + node_off);
    btype.insert(btype.end(), m.bface_type, m.bface_type + m.n_bfaces);
    bdata.insert(bdata.end(), m.bface_data, m.bface_data + m.n_bfaces * 8);
    W.insert(W.end(), W0[k], W0[k] + m.n_cells * nw);
    dt_field(&params[k], dim, m.n_cells, W0[k], Wdt);
    node_off += m.n_nodes;
    case_cell.push_back(case_cell.back() + m.n_cells);
    case_bface.push_back(case_bface.back() + m.n_bfaces);
    seeds.push_back(params[k].seed);
    case_row(&params[k], &cpar[static_cast<size_t>(k) * kCaseN]);
  }
  ugkwp_mesh u{};
  u.dim = dim;
  u.n_nodes = node_off;
  u.nodes = nodes.data();
  u.n_cells = case_cell.back();
  u.cell_ptr = cell_ptr.data();
  u.cell_nodes = cell_nodes.data();
  u.n_bfaces = case_bface.back();
  u.bface_nodes = bnodes.data();
  u.bface_type = btype.data();
  u.bface_data = bdata.data();
  ugkwp_params pu = p0;
  pu.particle_capacity = 0;
  for (int k = 0; k < n_cases; ++k) pu.particle_capacity += params[k].particle_capacity;
  return init_impl(c, &u, &pu, W.data(), Wdt.data(), n_cases, case_cell, case_bface, seeds, cpar);
}

}  // extern "C"

namespace {

// Sizes the store and the particle-parallel grids for steps whose
// pre-transport set is about `need` particles, `need_new` of them new.
int plan_launches(ugkwp_ctx *c, int64_t need, int64_t need_new) {
  // without allocation the store stays as it is; a step that does not fit
  // halts in k_check and fails (run_steps)
  if (c->noalloc) need = std::min(need, c->cap);
  int rc = ensure_capacity(c, need);
  if (rc) return rc;
  // rounded up so that the launch arguments, and a captured graph, stay the
  // same from batch to batch while the counts fluctuate
  const int64_t q = int64_t{1} << 17, qn = int64_t{1} << 14;
  c->cover = std::min<int64_t>(c->cap, (need + need / 8 + 65536 + q - 1) / q * q);
  c->cover_new = (need_new + need_new / 8 + 16384 + qn - 1) / qn * qn;
  c->est_total = std::max<int64_t>(c->last_total, 1);
  c->est_new = std::max<int64_t>(c->last_new, 1);
  c->est_kept = std::max<int64_t>(c->n_ret, 1);
  return UGKWP_OK;
}

void drop_graph(ugkwp_ctx *c) {
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  c->gexec = nullptr;
  c->graph = nullptr;
  c->gkey.clear();
}

// The launch arguments a two-step graph bakes in: buffer addresses (they
// change when the store grows), capacity, grid coverage and tuning.
std::vector<int64_t> graph_key(const ugkwp_ctx *c) {
  return {reinterpret_cast<int64_t>(c->A.x), reinterpret_cast<int64_t>(c->B.x), reinterpret_cast<int64_t>(c->A32.x),
          reinterpret_cast<int64_t>(c->B32.x), reinterpret_cast<int64_t>(c->S.Sret), reinterpret_cast<int64_t>(c->S.tghost),
          reinterpret_cast<int64_t>(c->T.x), reinterpret_cast<int64_t>(c->T32.x), c->cap, c->cover, c->cover_new,
          c->transport_block, c->shakhov_lanes, c->P.max_cross, c->xw_exp, c->xm_exp, c->xr_exp,
          c->scatter_block, c->tally_block, c->flux_block};
}

// Captures two steps into a graph (the double-buffer swaps of two steps
// leave every pointer as it was, so the graph can be replayed), unless one
// with the same arguments exists.  The step sequence has no memset nodes.
int ensure_graph(ugkwp_ctx *c) {
  const std::vector<int64_t> key = graph_key(c);
  if (c->gexec && key == c->gkey) return UGKWP_OK;
  drop_graph(c);
  HIPCHK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  int rc = enqueue(c);
  if (!rc) rc = enqueue(c);
  hipGraph_t gr = nullptr;
  const hipError_t e = hipStreamEndCapture(c->stream, &gr);
  if (rc) {
    if (gr) (void)hipGraphDestroy(gr);
    return rc;
  }
  if (e != hipSuccess) return set_err(c, UGKWP_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
  c->graph = gr;
  HIPCHK(hipGraphInstantiate(&c->gexec, gr, nullptr, nullptr, 0));
  c->gkey = key;
  return UGKWP_OK;
}

// Runs up to n_steps steps in batches; with `until`, stops after the step at
// which k_finish found the residual target met (*converged = 1).
int run_steps(ugkwp_ctx *c, int32_t n_steps, bool until, int32_t *converged) {
  if (converged) *converged = 0;
  int rc = sync_counts(c);
  if (rc) return rc;
  // the last pre-transport set with margin for growth over a batch
  rc = plan_launches(c, std::max(c->last_need, c->n_ret + std::max<int64_t>(2 * c->last_new, 4096) + c->last_new / 2),
                     std::max<int64_t>(c->last_need_new, 2 * c->last_new));
  if (rc) return rc;
  int32_t done = 0;
  while (done < n_steps) {
    const int32_t batch = std::min<int32_t>(n_steps - done, c->batch_steps);
    const int64_t step0 = c->step;
    int32_t k = 0;
    if (c->use_graph && !c->prof && !c->noalloc && batch >= 2) {
      rc = ensure_graph(c);
      if (rc) return rc;
      for (; k + 2 <= batch; k += 2) HIPCHK(hipGraphLaunch(c->gexec, c->stream));
    }
    for (; k < batch; ++k) {
      rc = enqueue(c);
      if (rc) return rc;
    }
    // one host synchronization per batch
    HIPCHK(hipMemcpyAsync(&c->pinned[0], c->S.dstep, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(&c->pinned[1], c->S.halt, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(&c->pinned[2], c->S.flags, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (c->prof) prof_harvest(c);
    const int64_t committed = c->pinned[0] - step0;
    if ((batch - committed) % 2 != 0) swap_buffers(c);  // halted steps did not advance the buffers
    c->step = c->pinned[0];
    done += static_cast<int32_t>(committed);
    const int halt = static_cast<int>(c->pinned[1] & 0xffffffff), flags = static_cast<int>(c->pinned[2] & 0xffffffff);
    rc = sync_counts(c);
    if (rc) return rc;
    if (flags & kFlagResidRange) {
      // a residual term outside its window: that step updated the fields and
      // is committed (later steps of the batch halted before changing anything)
      HIPCHK(hipMemsetAsync(c->S.halt, 0, sizeof(int), c->stream));
      HIPCHK(hipMemsetAsync(c->S.flags, 0, sizeof(int), c->stream));
      HIPCHK(hipStreamSynchronize(c->stream));
      return set_err(c, UGKWP_ENUMERIC, "a residual term outside its exact-summation window at step %lld",
                     (long long)(c->step - 1));
    }
    if (halt && until && flags == kFlagConverged) {
      // the step that met the target is done; the rest of the batch was skipped
      HIPCHK(hipMemsetAsync(c->S.halt, 0, sizeof(int), c->stream));
      HIPCHK(hipMemsetAsync(c->S.flags, 0, sizeof(int), c->stream));
      HIPCHK(hipStreamSynchronize(c->stream));
      if (converged) *converged = 1;
      return UGKWP_OK;
    }
    if (halt && (flags & ~(kFlagCapacity | kFlagGrid)) == 0) {
      if (c->noalloc && c->last_need > c->cap) {
        HIPCHK(hipMemsetAsync(c->S.halt, 0, sizeof(int), c->stream));
        HIPCHK(hipMemsetAsync(c->S.flags, 0, sizeof(int), c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        return set_err(c, UGKWP_EOVERFLOW,
                       "step %lld needs %lld particle slots, the store holds %lld: ugkwp_step_noalloc does not grow it",
                       (long long)c->step, (long long)c->last_need, (long long)c->cap);
      }
      // the step was not committed: grow the store or the grids to its
      // recorded bounds and resume from it
      rc = plan_launches(c, c->last_need + c->last_need / 4 + 4096, c->last_need_new + c->last_need_new / 4);
      if (rc) return rc;
      HIPCHK(hipMemsetAsync(c->S.halt, 0, sizeof(int), c->stream));
      HIPCHK(hipMemsetAsync(c->S.flags, 0, sizeof(int), c->stream));
      continue;
    }
    if (halt) {
      // the failed step was not committed: fields, particles, tallies,
      // averages and the step counter are those of the last committed step,
      // and the context can be used on
      HIPCHK(hipMemsetAsync(c->S.halt, 0, sizeof(int), c->stream));
      HIPCHK(hipMemsetAsync(c->S.flags, 0, sizeof(int), c->stream));
      HIPCHK(hipStreamSynchronize(c->stream));
      if (flags & kFlagInvalid) return set_err(c, UGKWP_ENUMERIC, "invalid cell state at step %lld", (long long)c->step);
      if (flags & kFlagRunaway)
        return set_err(c, UGKWP_ENUMERIC, "runaway particle tracking at step %lld", (long long)c->step);
      if (flags & kFlagOverflow) return set_err(c, UGKWP_EOVERFLOW, "more than 2^20 particles in one cell");
      if (flags & kFlagRange)
        return set_err(c, UGKWP_ENUMERIC, "a tally term outside its exact-summation window at step %lld",
                       (long long)c->step);
      return set_err(c, UGKWP_EDEVICE, "step halted (flags %d)", flags);
    }
    // room for the next batch
    rc = plan_launches(c, std::max(c->last_need, c->n_ret + std::max<int64_t>(2 * c->last_new, 4096) + c->last_new / 2),
                       std::max<int64_t>(c->last_need_new, 2 * c->last_new));
    if (rc) return rc;
  }
  return UGKWP_OK;
}

}  // namespace

extern "C" {

int ugkwp_step(ugkwp_ctx *c, int32_t n_steps) {
  if (!c || n_steps < 0) return UGKWP_EINVAL;
  if (!c->S.W) return set_err(c, UGKWP_ESTATE, "context not initialized");
  if (c->step + n_steps >= (1 << 20) - 1) return set_err(c, UGKWP_EOVERFLOW, "step count exceeds the pid layout (2^20)");
  return run_steps(c, n_steps, false, nullptr);
}

int ugkwp_step_noalloc(ugkwp_ctx *c, int32_t n_steps) {
  if (!c || n_steps < 0) return UGKWP_EINVAL;
  if (!c->S.W) return set_err(c, UGKWP_ESTATE, "context not initialized");
  if (c->step + n_steps >= (1 << 20) - 1) return set_err(c, UGKWP_EOVERFLOW, "step count exceeds the pid layout (2^20)");
  if (c->prof) return set_err(c, UGKWP_ESTATE, "per-kernel timing creates events: switch it off first");
  if (!c->noalloc_scratch) return set_err(c, UGKWP_EDEVICE, "no scratch array");
  // layout of the step's accumulators in the scratch array (256-byte aligned)
  const int64_t nc = c->nc, nb1 = std::max<int64_t>(c->nb, 1);
  const int64_t scan_blocks = std::max<int64_t>(1, (std::max(2 * nc, nc + c->nb) + kScanBlock) / kScanBlock) + 1;
  size_t at = 0;
  auto take = [&](size_t bytes) {
    const size_t o = at;
    at += (bytes + 255) / 256 * 256;
    return o;
  };
  const size_t o_count = take(2 * nc * sizeof(int)), o_cursor = take(2 * nc * sizeof(int64_t)),
               o_wimp = take(nb1 * 3 * kTallyLimbs * sizeof(double)), o_resid = take(8 * c->ncase * sizeof(double)),
               o_nghost = take(sizeof(int64_t)), o_stats = take(kStatSlots * kStatN * sizeof(int64_t)),
               o_scan = take(scan_blocks * sizeof(int64_t));
  if (at > kNoAllocScratchBytes)
    return set_err(c, UGKWP_EOVERFLOW, "the step's accumulators need %zu bytes, the scratch array holds %zu", at,
                   kNoAllocScratchBytes);
  unsigned char *base = c->noalloc_scratch;
  State saved = c->S;
  int64_t *saved_scan = c->scan_tmp;
  const int64_t saved_scan_n = c->scan_tmp_n;
  c->S.count = reinterpret_cast<int *>(base + o_count);
  c->S.cursor = reinterpret_cast<int64_t *>(base + o_cursor);
  c->S.wimp = reinterpret_cast<double *>(base + o_wimp);
  c->S.resid = reinterpret_cast<double *>(base + o_resid);
  c->S.nghost = reinterpret_cast<int64_t *>(base + o_nghost);
  c->S.stats = reinterpret_cast<int64_t *>(base + o_stats);
  c->scan_tmp = reinterpret_cast<int64_t *>(base + o_scan);
  c->scan_tmp_n = scan_blocks;
  c->noalloc = true;
  const int rc = run_steps(c, n_steps, false, nullptr);
  (void)hipStreamSynchronize(c->stream);
  c->noalloc = false;
  // the pointers that the double buffering swaps (tallies, offsets) stay as
  // the steps left them; the scratch pointers go back to the context's own
  c->S.count = saved.count;
  c->S.cursor = saved.cursor;
  c->S.wimp = saved.wimp;
  c->S.resid = saved.resid;
  c->S.nghost = saved.nghost;
  c->S.stats = saved.stats;
  c->scan_tmp = saved_scan;
  c->scan_tmp_n = saved_scan_n;
  return rc;
}

int ugkwp_step_until(ugkwp_ctx *c, double target, int32_t max_steps, int32_t *converged) {
  if (!c || max_steps < 0 || !(target > 0.0) || !converged) return UGKWP_EINVAL;
  if (!c->S.W) return set_err(c, UGKWP_ESTATE, "context not initialized");
  if (c->step + max_steps >= (1 << 20) - 1) return set_err(c, UGKWP_EOVERFLOW, "step count exceeds the pid layout (2^20)");
  HIPCHK(hipMemcpyAsync(c->S.scal + kScalTarget, &target, sizeof(double), hipMemcpyHostToDevice, c->stream));
  const int rc = run_steps(c, max_steps, true, converged);
  const double off = 0.0;
  HIPCHK(hipMemcpyAsync(c->S.scal + kScalTarget, &off, sizeof(double), hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return rc;
}

int ugkwp_residual(ugkwp_ctx *c, double *r_inst, double *r_avg, int64_t *step) {
  if (!c) return UGKWP_EINVAL;
  std::vector<double> s(c->ncase * kScalN);
  HIPCHK(hipMemcpyAsync(s.data(), c->S.scal, s.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  double ri = 0.0, ra = 0.0;
  for (int k = 0; k < c->ncase; ++k) {
    ri = std::max(ri, s[k * kScalN + kScalRinst]);
    ra = std::max(ra, s[k * kScalN + kScalRavg]);
  }
  if (r_inst) *r_inst = ri;
  if (r_avg) *r_avg = ra;
  if (step) *step = c->step;
  return UGKWP_OK;
}

int ugkwp_case_residual(ugkwp_ctx *c, int32_t case_id, double *r_inst, double *r_avg) {
  if (!c || case_id < 0 || case_id >= c->ncase) return UGKWP_EINVAL;
  double s[kScalN];
  HIPCHK(hipMemcpyAsync(s, c->S.scal + case_id * kScalN, sizeof s, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  if (r_inst) *r_inst = s[kScalRinst];
  if (r_avg) *r_avg = s[kScalRavg];
  return UGKWP_OK;
}

int ugkwp_case_range(ugkwp_ctx *c, int32_t case_id, int64_t *first_cell, int64_t *n_cells, int64_t *first_wall,
                     int64_t *n_wall) {
  if (!c || case_id < 0 || case_id >= c->ncase) return UGKWP_EINVAL;
  if (first_cell) *first_cell = c->h_case_cell[case_id];
  if (n_cells) *n_cells = c->h_case_cell[case_id + 1] - c->h_case_cell[case_id];
  // wall faces are listed in boundary-face order, so a case's are contiguous
  int64_t w0 = 0, w1 = 0;
  for (int64_t k = 0; k < c->nwall; ++k) {
    const int b = c->h_wall_b[k];
    if (b < c->h_case_bface[case_id]) w0 = k + 1;
    if (b < c->h_case_bface[case_id + 1]) w1 = k + 1;
  }
  if (first_wall) *first_wall = w0;
  if (n_wall) *n_wall = w1 - w0;
  return UGKWP_OK;
}

int ugkwp_case_surface(ugkwp_ctx *c, int32_t case_id, int32_t mode, double *out, int64_t cap, int64_t *n_wall,
                       double *Cd) {
  if (!c || mode < 0 || mode > 2 || case_id < 0 || case_id >= c->ncase) return UGKWP_EINVAL;
  int64_t w0 = 0, nwc = 0;
  ugkwp_case_range(c, case_id, nullptr, nullptr, &w0, &nwc);
  if (n_wall) *n_wall = nwc;
  if (c->step == 0) return set_err(c, UGKWP_ESTATE, "no step done yet");
  double s[kScalN];
  HIPCHK(hipMemcpyAsync(s, c->S.scal + case_id * kScalN, sizeof s, hipMemcpyDeviceToHost, c->stream));
  std::vector<double> w(std::max<int64_t>(nwc, 1) * 3);
  const double *src = mode == 0 ? c->S.wlast : mode == 1 ? c->S.wsum : c->S.wema;
  if (nwc > 0)
    HIPCHK(hipMemcpyAsync(w.data(), src + 3 * w0, nwc * 3 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  if (Cd) *Cd = mode == 0 ? s[kScalCdLast] : mode == 1 ? s[kScalCdSum] / static_cast<double>(c->step) : s[kScalCdEma];
  if (!out) return UGKWP_OK;
  if (cap < nwc) return set_err(c, UGKWP_EOVERFLOW, "surface buffer too small");
  const double *cp = &c->h_case_par[static_cast<size_t>(case_id) * kCaseN];
  const double rho_inf = cp[kCaseRho], U = cp[kCaseU];
  const double qd = 0.5 * rho_inf * U * U;
  const double pinf = rho_inf * c->P.R * cp[kCaseT];
  const double scale = mode == 1 ? 1.0 / static_cast<double>(c->step) : 1.0;
  for (int64_t q = 0; q < nwc; ++q) {
    const int64_t k = w0 + q;
    const int b = c->h_wall_b[k];
    const int64_t l = static_cast<int64_t>(c->h_bcell[b]) * c->NV + c->h_bk[b];
    const int fs = c->h_lface[l];
    const int f = fs >= 0 ? fs : ~fs;
    out[6 * q + 0] = c->h_face_mid[2 * f];
    out[6 * q + 1] = c->h_face_mid[2 * f + 1];
    out[6 * q + 2] = c->h_lfn[l * 4 + 3];
    out[6 * q + 3] = (w[3 * q] * scale - pinf) / qd;
    out[6 * q + 4] = w[3 * q + 1] * scale / qd;
    out[6 * q + 5] = w[3 * q + 2] * scale / (qd * U);
  }
  return UGKWP_OK;
}

int ugkwp_surface(ugkwp_ctx *c, int32_t mode, double *out, int64_t cap, int64_t *n_wall, double *Cd) {
  return ugkwp_case_surface(c, 0, mode, out, cap, n_wall, Cd);
}

int ugkwp_get_fields(ugkwp_ctx *c, double *W) {
  if (!c || !W) return UGKWP_EINVAL;
  HIPCHK(hipMemcpyAsync(W, c->S.W, c->nc * c->nw * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return UGKWP_OK;
}

int ugkwp_get_fields_device(ugkwp_ctx *c, void *d_W) {
  if (!c || !d_W) return UGKWP_EINVAL;
  HIPCHK(hipMemcpyAsync(d_W, c->S.W, c->nc * c->nw * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  return UGKWP_OK;
}

int ugkwp_get_dt(ugkwp_ctx *c, double *dt) {
  if (!c || !dt) return UGKWP_EINVAL;
  HIPCHK(hipMemcpyAsync(dt, c->S.dt, c->nc * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return UGKWP_OK;
}

int ugkwp_get_counts(ugkwp_ctx *c, int32_t *count, int64_t *n_total, int64_t *n_new, int64_t *n_removed,
                     int64_t *n_exited, int64_t *n_guard) {
  if (!c) return UGKWP_EINVAL;
  // committed values only: the retained set's offsets and the last
  // committed step's counts
  int64_t info[kInfoN];
  std::vector<int64_t> off(count ? c->nc + 1 : 0);
  if (count) HIPCHK(hipMemcpyAsync(off.data(), c->S.roff, (c->nc + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipMemcpyAsync(info, c->S.info, sizeof info, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  if (count)
    for (int64_t i = 0; i < c->nc; ++i) count[i] = static_cast<int32_t>(off[i + 1] - off[i]);
  if (n_total) *n_total = info[kInfoTotal];
  if (n_new) *n_new = info[kInfoNew];
  if (n_removed) *n_removed = info[kInfoRemoved];
  if (n_exited) *n_exited = info[kInfoExited];
  if (n_guard) *n_guard = info[kInfoGuard];
  return UGKWP_OK;
}

int ugkwp_get_shakhov_fallbacks(ugkwp_ctx *c, int64_t *n_capped) {
  if (!c || !n_capped) return UGKWP_EINVAL;
  int64_t info[kInfoN];
  HIPCHK(hipMemcpyAsync(info, c->S.info, sizeof info, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  *n_capped = info[kInfoCapped];
  return UGKWP_OK;
}

int ugkwp_get_work(ugkwp_ctx *c, int64_t *n_transported) {
  if (!c || !n_transported) return UGKWP_EINVAL;
  int64_t info[kInfoN];
  HIPCHK(hipMemcpyAsync(info, c->S.info, sizeof info, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  *n_transported = info[kInfoSumTotal];
  return UGKWP_OK;
}

}  // extern "C"

namespace {

// Reads the first n slots of a store to host arrays in FP64 with global
// positions (the FP32 store holds positions relative to the cell anchor).
template <class R>
int read_store(ugkwp_ctx *c, const StoreT<R> &s, int64_t n, std::vector<uint64_t> &P, std::vector<int> &C,
               std::vector<double> &X, std::vector<double> &Y, std::vector<double> &U0, std::vector<double> &U1,
               std::vector<double> &U2, std::vector<double> &M, std::vector<double> &EI) {
  std::vector<R> x(n), y(c->dim == 2 ? n : 0), u0(n), u1(n), u2(n), ei(s.ei ? n : 0);
  if (n > 0) {
    HIPCHK(hipMemcpyAsync(P.data(), s.pid, n * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(C.data(), s.cell, n * 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(x.data(), s.x, n * sizeof(R), hipMemcpyDeviceToHost, c->stream));
    if (c->dim == 2) HIPCHK(hipMemcpyAsync(y.data(), s.y, n * sizeof(R), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(u0.data(), s.ux, n * sizeof(R), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(u1.data(), s.uy, n * sizeof(R), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(u2.data(), s.uz, n * sizeof(R), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(M.data(), s.m, n * 8, hipMemcpyDeviceToHost, c->stream));
    if (s.ei) HIPCHK(hipMemcpyAsync(ei.data(), s.ei, n * sizeof(R), hipMemcpyDeviceToHost, c->stream));
  }
  HIPCHK(hipStreamSynchronize(c->stream));
  const bool rel = c->precision != 0;
  for (int64_t k = 0; k < n; ++k) {
    const double ax = rel ? c->h_anchor[2 * C[k]] : 0.0, ay = rel ? c->h_anchor[2 * C[k] + 1] : 0.0;
    X[k] = rel ? ax + static_cast<double>(x[k]) : static_cast<double>(x[k]);
    if (c->dim == 2) Y[k] = rel ? ay + static_cast<double>(y[k]) : static_cast<double>(y[k]);
    U0[k] = u0[k];
    U1[k] = u1[k];
    U2[k] = u2[k];
    EI[k] = s.ei ? static_cast<double>(ei[k]) : 0.0;
  }
  return UGKWP_OK;
}

// Writes host arrays (FP64, global positions) to the first n slots.
template <class R>
int write_store(ugkwp_ctx *c, const StoreT<R> &s, int64_t n, const std::vector<uint64_t> &P,
                const std::vector<int> &C, const std::vector<double> &X, const std::vector<double> &Y,
                const std::vector<double> &U0, const std::vector<double> &U1, const std::vector<double> &U2,
                const std::vector<double> &M, const std::vector<double> &EI) {
  std::vector<R> x(n), y(n), u0(n), u1(n), u2(n), ei(n);
  const bool rel = c->precision != 0;
  for (int64_t k = 0; k < n; ++k) {
    const double ax = rel ? c->h_anchor[2 * C[k]] : 0.0, ay = rel ? c->h_anchor[2 * C[k] + 1] : 0.0;
    x[k] = static_cast<R>(rel ? X[k] - ax : X[k]);
    y[k] = static_cast<R>(rel ? Y[k] - ay : Y[k]);
    u0[k] = static_cast<R>(U0[k]);
    u1[k] = static_cast<R>(U1[k]);
    u2[k] = static_cast<R>(U2[k]);
    ei[k] = static_cast<R>(EI[k]);
  }
  const hipMemcpyKind h2d = hipMemcpyHostToDevice;
  if (n > 0) {
    HIPCHK(hipMemcpyAsync(s.pid, P.data(), n * 8, h2d, c->stream));
    HIPCHK(hipMemcpyAsync(s.cell, C.data(), n * 4, h2d, c->stream));
    HIPCHK(hipMemcpyAsync(s.x, x.data(), n * sizeof(R), h2d, c->stream));
    if (c->dim == 2) HIPCHK(hipMemcpyAsync(s.y, y.data(), n * sizeof(R), h2d, c->stream));
    HIPCHK(hipMemcpyAsync(s.ux, u0.data(), n * sizeof(R), h2d, c->stream));
    HIPCHK(hipMemcpyAsync(s.uy, u1.data(), n * sizeof(R), h2d, c->stream));
    HIPCHK(hipMemcpyAsync(s.uz, u2.data(), n * sizeof(R), h2d, c->stream));
    HIPCHK(hipMemcpyAsync(s.m, M.data(), n * 8, h2d, c->stream));
    if (s.ei) HIPCHK(hipMemcpyAsync(s.ei, ei.data(), n * sizeof(R), h2d, c->stream));
  }
  HIPCHK(hipStreamSynchronize(c->stream));
  return UGKWP_OK;
}

}  // namespace

extern "C" {

int ugkwp_get_particles(ugkwp_ctx *c, int64_t cap, uint64_t *pid, int32_t *cell, double *m, double *x, double *u,
                        double *ei, int64_t *n) {
  if (!c || !n) return UGKWP_EINVAL;
  const int64_t np = c->n_ret;
  *n = np;
  if (cap < np) return set_err(c, UGKWP_EOVERFLOW, "particle buffer too small");
  std::vector<uint64_t> P(np);
  std::vector<int> C(np);
  std::vector<double> X(np), Y(c->dim == 2 ? np : 0), U0(np), U1(np), U2(np), M(np), EI(np);
  const int rc = c->precision ? read_store(c, c->A32, np, P, C, X, Y, U0, U1, U2, M, EI)
                              : read_store(c, c->A, np, P, C, X, Y, U0, U1, U2, M, EI);
  if (rc) return rc;
  std::vector<int64_t> order(np);
  for (int64_t k = 0; k < np; ++k) order[k] = k;
  // by pid, then cell: the cases of a batch number their particles each on their own
  std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return P[a] != P[b] ? P[a] < P[b] : C[a] < C[b]; });
  for (int64_t j = 0; j < np; ++j) {
    const int64_t k = order[j];
    if (pid) pid[j] = P[k];
    if (cell) cell[j] = C[k];
    if (m) m[j] = M[k];
    if (x) {
      x[j * c->dim] = X[k];
      if (c->dim == 2) x[j * 2 + 1] = Y[k];
    }
    if (u) {
      u[3 * j] = U0[k];
      u[3 * j + 1] = U1[k];
      u[3 * j + 2] = U2[k];
    }
    if (ei) ei[j] = EI[k];
  }
  return UGKWP_OK;
}

int ugkwp_set_particles(ugkwp_ctx *c, int64_t n, const uint64_t *pid, const int32_t *cell, const double *m,
                        const double *x, const double *u, const double *ei) {
  if (!c || n < 0 || (n > 0 && (!pid || !cell || !m || !x || !u))) return UGKWP_EINVAL;
  std::vector<int64_t> order(n);
  for (int64_t k = 0; k < n; ++k) {
    if (cell[k] < 0 || cell[k] >= c->nc) return set_err(c, UGKWP_EINVAL, "particle cell out of range");
    order[k] = k;
  }
  std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
    return cell[a] != cell[b] ? cell[a] < cell[b] : pid[a] < pid[b];
  });
  int rc = ensure_capacity(c, n);
  if (rc) return rc;
  std::vector<uint64_t> P(n);
  std::vector<int> C(n);
  std::vector<double> X(n), Y(n), U0(n), U1(n), U2(n), M(n), EI(n, 0.0);
  std::vector<int64_t> ro(2 * c->nc + 1, 0);
  for (int64_t j = 0; j < n; ++j) {
    const int64_t k = order[j];
    P[j] = pid[k];
    C[j] = cell[k];
    M[j] = m[k];
    X[j] = x[k * c->dim];
    Y[j] = c->dim == 2 ? x[k * 2 + 1] : 0.0;
    U0[j] = u[3 * k];
    U1[j] = u[3 * k + 1];
    U2[j] = u[3 * k + 2];
    if (ei && c->P.D > 0) EI[j] = ei[k];
    ro[C[j] + 1]++;
  }
  for (int64_t i = 0; i < c->nc; ++i) ro[i + 1] += ro[i];
  for (int64_t i = c->nc + 1; i <= 2 * c->nc; ++i) ro[i] = n;  // no collided particles
  rc = c->precision ? write_store(c, c->A32, n, P, C, X, Y, U0, U1, U2, M, EI)
                    : write_store(c, c->A, n, P, C, X, Y, U0, U1, U2, M, EI);
  if (rc) return rc;
  HIPCHK(hipMemcpyAsync(c->S.roff, ro.data(), ro.size() * 8, hipMemcpyHostToDevice, c->stream));
  // the retained tally W^p Omega (and the raw moments) from the store as the
  // device holds it: the same exact sums a step computes
  const Geo g = c->geo();
  if (c->precision) {
    if (c->dim == 1) launch_tally<1, float>(c, g, c->A32, c->S.roff, c->S.Sret, c->S.Xret, nullptr, c->S.Mraw);
    else launch_tally<2, float>(c, g, c->A32, c->S.roff, c->S.Sret, c->S.Xret, nullptr, c->S.Mraw);
  } else {
    if (c->dim == 1) launch_tally<1, double>(c, g, c->A, c->S.roff, c->S.Sret, c->S.Xret, nullptr, c->S.Mraw);
    else launch_tally<2, double>(c, g, c->A, c->S.roff, c->S.Sret, c->S.Xret, nullptr, c->S.Mraw);
  }
  HIPCHK(hipGetLastError());
  c->n_ret = n;
  rc = check_flags(c);
  if (rc) return rc;
  return UGKWP_OK;
}

int ugkwp_set_fields(ugkwp_ctx *c, const double *W) {
  if (!c || !W) return UGKWP_EINVAL;
  std::vector<double> r(c->nc);
  for (int64_t i = 0; i < c->nc; ++i) r[i] = W[i * c->nw];
  HIPCHK(hipMemcpyAsync(c->S.W, W, c->nc * c->nw * sizeof(double), hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(c->S.rho_prev, r.data(), c->nc * sizeof(double), hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return UGKWP_OK;
}

int ugkwp_set_step(ugkwp_ctx *c, int64_t step) {
  if (!c || step < 0 || step >= (1 << 20)) return UGKWP_EINVAL;
  HIPCHK(hipMemcpyAsync(c->S.dstep, &step, sizeof(int64_t), hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  c->step = step;
  return UGKWP_OK;
}

int ugkwp_get_face_flux(ugkwp_ctx *c, double *Fs, int64_t cap, int64_t *n_faces) {
  if (!c) return UGKWP_EINVAL;
  if (n_faces) *n_faces = c->nf;
  if (!Fs) return UGKWP_OK;
  if (cap < c->nf) return set_err(c, UGKWP_EOVERFLOW, "face buffer too small");
  HIPCHK(hipMemcpyAsync(Fs, c->Fs_prev, c->nf * c->nw * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return UGKWP_OK;
}

int ugkwp_get_history(ugkwp_ctx *c, double *rho_prev, double *rho_sum, double *rho_mean_prev, double *wlast,
                      double *wsum, double *wema, double *scal) {
  if (!c) return UGKWP_EINVAL;
  const size_t nc = c->nc * sizeof(double), nw3 = c->nwall * 3 * sizeof(double);
  const hipMemcpyKind d2h = hipMemcpyDeviceToHost;
  if (rho_prev) HIPCHK(hipMemcpyAsync(rho_prev, c->S.rho_prev, nc, d2h, c->stream));
  if (rho_sum) HIPCHK(hipMemcpyAsync(rho_sum, c->S.rho_sum, nc, d2h, c->stream));
  if (rho_mean_prev) HIPCHK(hipMemcpyAsync(rho_mean_prev, c->S.rho_mean_prev, nc, d2h, c->stream));
  if (wlast && nw3) HIPCHK(hipMemcpyAsync(wlast, c->S.wlast, nw3, d2h, c->stream));
  if (wsum && nw3) HIPCHK(hipMemcpyAsync(wsum, c->S.wsum, nw3, d2h, c->stream));
  if (wema && nw3) HIPCHK(hipMemcpyAsync(wema, c->S.wema, nw3, d2h, c->stream));
  if (scal) HIPCHK(hipMemcpyAsync(scal, c->S.scal, c->ncase * kScalN * sizeof(double), d2h, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  if (scal)
    for (int k = 0; k < c->ncase; ++k) scal[k * kScalN + kScalTarget] = 0.0;
  return UGKWP_OK;
}

int ugkwp_set_history(ugkwp_ctx *c, const double *rho_prev, const double *rho_sum, const double *rho_mean_prev,
                      const double *wlast, const double *wsum, const double *wema, const double *scal) {
  if (!c) return UGKWP_EINVAL;
  const size_t nc = c->nc * sizeof(double), nw3 = c->nwall * 3 * sizeof(double);
  const hipMemcpyKind h2d = hipMemcpyHostToDevice;
  std::vector<double> sc;
  if (scal) {
    sc.assign(scal, scal + c->ncase * kScalN);
    for (int k = 0; k < c->ncase; ++k) sc[k * kScalN + kScalTarget] = 0.0;
  }
  if (rho_prev) HIPCHK(hipMemcpyAsync(c->S.rho_prev, rho_prev, nc, h2d, c->stream));
  if (rho_sum) HIPCHK(hipMemcpyAsync(c->S.rho_sum, rho_sum, nc, h2d, c->stream));
  if (rho_mean_prev) HIPCHK(hipMemcpyAsync(c->S.rho_mean_prev, rho_mean_prev, nc, h2d, c->stream));
  if (wlast && nw3) HIPCHK(hipMemcpyAsync(c->S.wlast, wlast, nw3, h2d, c->stream));
  if (wsum && nw3) HIPCHK(hipMemcpyAsync(c->S.wsum, wsum, nw3, h2d, c->stream));
  if (wema && nw3) HIPCHK(hipMemcpyAsync(c->S.wema, wema, nw3, h2d, c->stream));
  if (scal) HIPCHK(hipMemcpyAsync(c->S.scal, sc.data(), sc.size() * sizeof(double), h2d, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return UGKWP_OK;
}

}  // extern "C"

namespace {

// Checkpoint file: a fixed header, then the arrays in this order (native
// byte order): W, dt, rho_prev, rho_sum, rho_mean_prev, wlast, wsum, wema,
// scal, info, and the committed particle store as the device holds it (its
// order and, for the FP32 store, its cell-relative positions): x, (y), ux,
// uy, uz, (ei) in the store's type, m, pid, cell.
constexpr char kSaveMagic[8] = {'U', 'G', 'K', 'W', 'P', 'S', 'V', '1'};
struct SaveHeader {
  char magic[8];
  int32_t version, dim, precision, D, ncase, xw, xm, xr;
  int64_t nc, nb, nwall, nf, n_ret, step;
  uint64_t seed;
};

struct File {
  FILE *f = nullptr;
  ~File() {
    if (f) fclose(f);
  }
};

template <class T>
bool fput(FILE *f, const T *p, size_t n) {
  return n == 0 || fwrite(p, sizeof(T), n, f) == n;
}
template <class T>
bool fget(FILE *f, T *p, size_t n) {
  return n == 0 || fread(p, sizeof(T), n, f) == n;
}

template <class T>
int d2h(ugkwp_ctx *c, std::vector<T> &h, const T *d, size_t n) {
  h.resize(n);
  if (n) HIPCHK(hipMemcpyAsync(h.data(), d, n * sizeof(T), hipMemcpyDeviceToHost, c->stream));
  return UGKWP_OK;
}
template <class T>
int h2d(ugkwp_ctx *c, T *d, const std::vector<T> &h) {
  if (!h.empty()) HIPCHK(hipMemcpyAsync(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, c->stream));
  return UGKWP_OK;
}

template <class R>
int save_store(ugkwp_ctx *c, const StoreT<R> &s, FILE *f) {
  const size_t n = c->n_ret;
  std::vector<R> x, y, u0, u1, u2, ei;
  std::vector<double> m;
  std::vector<uint64_t> pid;
  std::vector<int> cell;
  d2h(c, x, s.x, n);
  if (c->dim == 2) d2h(c, y, s.y, n);
  d2h(c, u0, s.ux, n);
  d2h(c, u1, s.uy, n);
  d2h(c, u2, s.uz, n);
  if (s.ei) d2h(c, ei, s.ei, n);
  d2h(c, m, s.m, n);
  d2h(c, pid, s.pid, n);
  d2h(c, cell, s.cell, n);
  HIPCHK(hipStreamSynchronize(c->stream));
  bool ok = fput(f, x.data(), n) && (c->dim != 2 || fput(f, y.data(), n)) && fput(f, u0.data(), n) &&
            fput(f, u1.data(), n) && fput(f, u2.data(), n) && (!s.ei || fput(f, ei.data(), n)) &&
            fput(f, m.data(), n) && fput(f, pid.data(), n) && fput(f, cell.data(), n);
  return ok ? UGKWP_OK : set_err(c, UGKWP_EIO, "write failed");
}

template <class R>
int load_store(ugkwp_ctx *c, const StoreT<R> &s, FILE *f, size_t n, std::vector<int> &cell) {
  std::vector<R> x(n), y(c->dim == 2 ? n : 0), u0(n), u1(n), u2(n), ei(s.ei ? n : 0);
  std::vector<double> m(n);
  std::vector<uint64_t> pid(n);
  cell.resize(n);
  bool ok = fget(f, x.data(), n) && (c->dim != 2 || fget(f, y.data(), n)) && fget(f, u0.data(), n) &&
            fget(f, u1.data(), n) && fget(f, u2.data(), n) && (!s.ei || fget(f, ei.data(), n)) &&
            fget(f, m.data(), n) && fget(f, pid.data(), n) && fget(f, cell.data(), n);
  if (!ok) return set_err(c, UGKWP_EIO, "checkpoint truncated");
  for (size_t k = 0; k < n; ++k)
    if (cell[k] < 0 || cell[k] >= c->nc || (k > 0 && cell[k] < cell[k - 1]))
      return set_err(c, UGKWP_EINVAL, "checkpoint particle cells out of range or not sorted");
  h2d(c, s.x, x);
  if (c->dim == 2) h2d(c, s.y, y);
  h2d(c, s.ux, u0);
  h2d(c, s.uy, u1);
  h2d(c, s.uz, u2);
  if (s.ei) h2d(c, s.ei, ei);
  h2d(c, s.m, m);
  h2d(c, s.pid, pid);
  h2d(c, s.cell, cell);
  HIPCHK(hipStreamSynchronize(c->stream));
  return UGKWP_OK;
}

}  // namespace

extern "C" {

int ugkwp_save(ugkwp_ctx *c, const char *path) {
  if (!c || !path) return UGKWP_EINVAL;
  if (!c->S.W) return set_err(c, UGKWP_ESTATE, "context not initialized");
  SaveHeader h{};
  memcpy(h.magic, kSaveMagic, 8);
  h.version = 1;
  h.dim = c->dim;
  h.precision = c->precision;
  h.D = c->P.D;
  h.ncase = c->ncase;
  h.xw = c->xw_exp;
  h.xm = c->xm_exp;
  h.xr = c->xr_exp;
  h.nc = c->nc;
  h.nb = c->nb;
  h.nwall = c->nwall;
  h.nf = c->nf;
  h.n_ret = c->n_ret;
  h.step = c->step;
  h.seed = c->P.seed;
  const size_t nc = c->nc, nw3 = c->nwall * 3;
  std::vector<double> W, dt, rp, rs, rm, wl, ws, we, sc;
  std::vector<int64_t> info;
  d2h(c, W, c->S.W, nc * c->nw);
  d2h(c, dt, c->S.dt, nc);
  d2h(c, rp, c->S.rho_prev, nc);
  d2h(c, rs, c->S.rho_sum, nc);
  d2h(c, rm, c->S.rho_mean_prev, nc);
  d2h(c, wl, c->S.wlast, nw3);
  d2h(c, ws, c->S.wsum, nw3);
  d2h(c, we, c->S.wema, nw3);
  d2h(c, sc, c->S.scal, c->ncase * kScalN);
  d2h(c, info, c->S.info, kInfoN);
  HIPCHK(hipStreamSynchronize(c->stream));
  for (int k = 0; k < c->ncase; ++k) sc[k * kScalN + kScalTarget] = 0.0;
  const std::string tmp = std::string(path) + ".tmp";
  {
    File F;
    F.f = fopen(tmp.c_str(), "wb");
    if (!F.f) return set_err(c, UGKWP_EIO, "cannot open %s for writing", tmp.c_str());
    bool ok = fput(F.f, &h, 1) && fput(F.f, W.data(), W.size()) && fput(F.f, dt.data(), nc) &&
              fput(F.f, rp.data(), nc) && fput(F.f, rs.data(), nc) && fput(F.f, rm.data(), nc) &&
              fput(F.f, wl.data(), nw3) && fput(F.f, ws.data(), nw3) && fput(F.f, we.data(), nw3) &&
              fput(F.f, sc.data(), sc.size()) && fput(F.f, info.data(), info.size());
    if (!ok) return set_err(c, UGKWP_EIO, "write failed");
    const int rc = c->precision ? save_store(c, c->A32, F.f) : save_store(c, c->A, F.f);
    if (rc) return rc;
    if (fflush(F.f) != 0) return set_err(c, UGKWP_EIO, "write failed");
  }
  if (std::rename(tmp.c_str(), path) != 0) return set_err(c, UGKWP_EIO, "cannot rename %s", tmp.c_str());
  return UGKWP_OK;
}

int ugkwp_load(ugkwp_ctx *c, const char *path) {
  if (!c || !path) return UGKWP_EINVAL;
  if (!c->S.W) return set_err(c, UGKWP_ESTATE, "context not initialized");
  File F;
  F.f = fopen(path, "rb");
  if (!F.f) return set_err(c, UGKWP_EIO, "cannot open %s", path);
  SaveHeader h{};
  if (!fget(F.f, &h, 1)) return set_err(c, UGKWP_EIO, "checkpoint truncated");
  if (memcmp(h.magic, kSaveMagic, 8) != 0 || h.version != 1) return set_err(c, UGKWP_EINVAL, "not a checkpoint");
  if (h.dim != c->dim || h.precision != c->precision || h.D != c->P.D || h.ncase != c->ncase || h.nc != c->nc ||
      h.nb != c->nb || h.nwall != c->nwall || h.nf != c->nf || h.n_ret < 0 || h.step < 0 || h.step >= (1 << 20))
    return set_err(c, UGKWP_EINVAL, "checkpoint does not match this context's mesh and parameters");
  const size_t nc = c->nc, nw3 = c->nwall * 3;
  std::vector<double> W(nc * c->nw), dt(nc), rp(nc), rs(nc), rm(nc), wl(nw3), ws(nw3), we(nw3),
      sc(c->ncase * kScalN);
  std::vector<int64_t> info(kInfoN);
  bool ok = fget(F.f, W.data(), W.size()) && fget(F.f, dt.data(), nc) && fget(F.f, rp.data(), nc) &&
            fget(F.f, rs.data(), nc) && fget(F.f, rm.data(), nc) && fget(F.f, wl.data(), nw3) &&
            fget(F.f, ws.data(), nw3) && fget(F.f, we.data(), nw3) && fget(F.f, sc.data(), sc.size()) &&
            fget(F.f, info.data(), info.size());
  if (!ok) return set_err(c, UGKWP_EIO, "checkpoint truncated");
  for (size_t i = 0; i < nc; ++i)
    if (!(dt[i] > 0.0) || !std::isfinite(dt[i])) return set_err(c, UGKWP_EINVAL, "checkpoint time steps invalid");
  HIPCHK(hipStreamSynchronize(c->stream));
  drop_graph(c);
  int rc = ensure_capacity(c, h.n_ret);
  if (rc) return rc;
  std::vector<int> cell;
  rc = c->precision ? load_store(c, c->A32, F.f, h.n_ret, cell) : load_store(c, c->A, F.f, h.n_ret, cell);
  if (rc) return rc;
  std::vector<int64_t> ro(2 * nc + 1, 0);
  for (int v : cell) ro[v + 1]++;
  for (size_t i = 0; i < nc; ++i) ro[i + 1] += ro[i];
  for (size_t i = nc + 1; i <= 2 * nc; ++i) ro[i] = h.n_ret;
  h2d(c, c->S.W, W);
  h2d(c, c->S.dt, dt);
  h2d(c, c->S.rho_prev, rp);
  h2d(c, c->S.rho_sum, rs);
  h2d(c, c->S.rho_mean_prev, rm);
  if (nw3) {
    h2d(c, c->S.wlast, wl);
    h2d(c, c->S.wsum, ws);
    h2d(c, c->S.wema, we);
  }
  h2d(c, c->S.scal, sc);
  h2d(c, c->S.info, info);
  h2d(c, c->S.roff, ro);
  const int64_t step = h.step;
  HIPCHK(hipMemcpyAsync(c->S.dstep, &step, sizeof step, hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipMemsetAsync(c->S.halt, 0, sizeof(int), c->stream));
  HIPCHK(hipMemsetAsync(c->S.flags, 0, sizeof(int), c->stream));
  c->xw_exp = h.xw;
  c->xm_exp = h.xm;
  c->xr_exp = h.xr;
  c->P.xw = make_window(h.xw, kTallyLimbs);
  c->P.xm = make_window(h.xm, kTallyLimbs);
  c->P.xr = make_window(h.xr, 4);
  // crossing ratios (and the FP32 tables) from the restored time steps
  Geo g = c->geo();
  hipLaunchKernelGGL(k_init_ratio, dim3(nblk(c->nc * c->NV, 256)), dim3(256), 0, c->stream, g, c->S.dt, c->lfn);
  if (c->precision)
    hipLaunchKernelGGL(k_init_mixed, dim3(nblk(c->nc * c->NV, 256)), dim3(256), 0, c->stream, g, c->lfn32, c->lda);
  c->n_ret = h.n_ret;
  c->step = h.step;
  if (c->precision) {
    if (c->dim == 1) launch_tally<1, float>(c, g, c->A32, c->S.roff, c->S.Sret, c->S.Xret, nullptr, c->S.Mraw);
    else launch_tally<2, float>(c, g, c->A32, c->S.roff, c->S.Sret, c->S.Xret, nullptr, c->S.Mraw);
  } else {
    if (c->dim == 1) launch_tally<1, double>(c, g, c->A, c->S.roff, c->S.Sret, c->S.Xret, nullptr, c->S.Mraw);
    else launch_tally<2, double>(c, g, c->A, c->S.roff, c->S.Sret, c->S.Xret, nullptr, c->S.Mraw);
  }
  HIPCHK(hipGetLastError());
  rc = check_flags(c);
  if (rc) return rc;
  return sync_counts(c);
}

int ugkwp_get_tally(ugkwp_ctx *c, double *Sminus, double *Splus) {
  if (!c) return UGKWP_EINVAL;
  const size_t bytes = c->nc * c->nw * sizeof(double);
  if (Sminus) HIPCHK(hipMemcpyAsync(Sminus, c->Sm_prev, bytes, hipMemcpyDeviceToHost, c->stream));
  if (Splus) HIPCHK(hipMemcpyAsync(Splus, c->Sp_prev, bytes, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return UGKWP_OK;
}

static bool block_ok(int32_t b) { return b == 64 || b == 128 || b == 256; }

int ugkwp_set_tuning(ugkwp_ctx *c, const ugkwp_tuning *t) {
  if (!c || !t) return UGKWP_EINVAL;
  if (t->batch_steps < 1 || t->batch_steps > 1024 || (t->use_graph != 0 && t->use_graph != 1) ||
      !block_ok(t->transport_block) || !(block_ok(t->scatter_block) || t->scatter_block == 512) ||
      !block_ok(t->tally_block) ||
      !block_ok(t->flux_block) ||
      (t->shakhov_lanes != 1 && t->shakhov_lanes != 2 && t->shakhov_lanes != 4 && t->shakhov_lanes != 8 &&
       t->shakhov_lanes != 16) ||
      t->max_crossings < 1 || t->max_crossings > 10000)
    return set_err(c, UGKWP_EINVAL, "tuning value out of range");
  c->batch_steps = t->batch_steps;
  c->use_graph = t->use_graph;
  c->transport_block = t->transport_block;
  c->shakhov_lanes = t->shakhov_lanes;
  c->max_crossings = t->max_crossings;
  c->P.max_cross = t->max_crossings;
  c->scatter_block = t->scatter_block;
  c->tally_block = t->tally_block;
  c->flux_block = t->flux_block;
  return UGKWP_OK;
}

int ugkwp_get_tuning(ugkwp_ctx *c, ugkwp_tuning *t) {
  if (!c || !t) return UGKWP_EINVAL;
  t->batch_steps = c->batch_steps;
  t->use_graph = c->use_graph;
  t->transport_block = c->transport_block;
  t->shakhov_lanes = c->shakhov_lanes;
  t->max_crossings = c->max_crossings;
  t->scatter_block = c->scatter_block;
  t->tally_block = c->tally_block;
  t->flux_block = c->flux_block;
  return UGKWP_OK;
}

int ugkwp_profile(ugkwp_ctx *c, int32_t enable) {
  if (!c) return UGKWP_EINVAL;
  HIPCHK(hipStreamSynchronize(c->stream));
  prof_harvest(c);
  if (enable) {
    for (int k = 0; k < kKCount; ++k) {
      c->prof_ms[k] = 0.0;
      c->prof_n[k] = 0;
      c->prof_bytes[k] = 0.0;
    }
  }
  c->prof = enable != 0;
  c->prof_all = enable == 1;
  return UGKWP_OK;
}

int ugkwp_stream_copy(void *dst, const void *src, int64_t bytes, int32_t reps, int32_t blocks, void *stream,
                      double *ms_per_copy) {
  const auto ad = reinterpret_cast<uintptr_t>(dst), as = reinterpret_cast<uintptr_t>(src);
  if (!dst || !src || bytes <= 0 || (bytes & 15) || (ad & 15) || (as & 15) || reps < 1 || blocks < 0 ||
      !ms_per_copy)
    return UGKWP_EINVAL;
  if ((ad < as + static_cast<uintptr_t>(bytes)) && (as < ad + static_cast<uintptr_t>(bytes))) return UGKWP_EINVAL;
  const int64_t n = bytes / 16;
  int grid = blocks;
  if (grid == 0) {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return UGKWP_EDEVICE;
    grid = 8 * cus;
  }
  const int64_t need = (n + 255) / 256;
  if (grid > need) grid = static_cast<int>(need);
  auto st = static_cast<hipStream_t>(stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess) return UGKWP_EDEVICE;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return UGKWP_EDEVICE;
  }
  bool ok = true;
  auto *d = static_cast<uint4 *>(dst);
  const auto *sp = static_cast<const uint4 *>(src);
  hipLaunchKernelGGL(k_stream_copy, dim3(grid), dim3(256), 0, st, d, sp, n);  // warm-up
  ok = ok && hipGetLastError() == hipSuccess && hipEventRecord(e0, st) == hipSuccess;
  for (int r = 0; ok && r < reps; ++r) {
    hipLaunchKernelGGL(k_stream_copy, dim3(grid), dim3(256), 0, st, d, sp, n);
    ok = hipGetLastError() == hipSuccess;
  }
  float ms = 0.0f;
  ok = ok && hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
       hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (!ok) return UGKWP_EDEVICE;
  *ms_per_copy = static_cast<double>(ms) / reps;
  return UGKWP_OK;
}

int ugkwp_profile_read(ugkwp_ctx *c, int32_t cap, const char **names, double *ms, int64_t *launches, double *bytes,
                       int32_t *n) {
  if (!c) return UGKWP_EINVAL;
  HIPCHK(hipStreamSynchronize(c->stream));
  prof_harvest(c);
  if (n) *n = kKCount;
  for (int k = 0; k < kKCount && k < cap; ++k) {
    if (names) names[k] = kKernelNames[k];
    if (ms) ms[k] = c->prof_ms[k];
    if (launches) launches[k] = c->prof_n[k];
    if (bytes) bytes[k] = c->prof_bytes[k];
  }
  return UGKWP_OK;
}

const char *ugkwp_last_error(const ugkwp_ctx *c) { return c ? c->err.c_str() : "no context"; }

void ugkwp_free(ugkwp_ctx *c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  drop_graph(c);
  for (auto &r : c->prof_pending) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : c->ev_pool) (void)hipEventDestroy(e);
  for (void *p : c->allocs) (void)hipFree(p);
  if (c->pinned) (void)hipHostFree(c->pinned);
  if (c->side) (void)hipStreamSynchronize(c->side);
  if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
  if (c->ev_join) (void)hipEventDestroy(c->ev_join);
  if (c->side) (void)hipStreamDestroy(c->side);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

}  // extern "C"
