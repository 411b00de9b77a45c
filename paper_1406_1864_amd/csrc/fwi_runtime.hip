// Host runtime of libfwi: validation, execution plans, workspace layout,
// batched time loops (direct launches or replayed hipGraph chunks), the
// autotuner and the C ABI of include/fwi.h.
//
// A plan fixes everything that depends only on the grid, the acquisition
// geometry and the execution settings: padded storage layout, the shot ->
// batch/slot schedule (shots sorted by record length, longest first), the
// per-shot descriptors (record length, snapshot spacing K = ceil(sqrt(nt)),
// source cell, receiver range, aperture), the receiver tile maps and the
// byte layout of the caller's workspace.  Plans are cached by a hash of
// those inputs; captured graphs are cached inside their plan, keyed by the
// device pointers they bake in.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/fwi.h"
#include "fwi_internal.h"

namespace fwi {
namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

#define HIP_TRY(expr)                                                               \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess)                                                           \
      return fail(FWI_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x, size_t a = kAlign) { return (x + a - 1) / a * a; }

// ---------------------------------------------------------------- hashing
struct Hasher {
  uint64_t h = 1469598103934665603ull;
  void bytes(const void* p, size_t n) {
    const unsigned char* c = (const unsigned char*)p;
    for (size_t i = 0; i < n; ++i) {
      h ^= c[i];
      h *= 1099511628211ull;
    }
  }
  template <class T>
  void pod(const T& v) { bytes(&v, sizeof(T)); }
  // field by field: the struct's padding bytes are not part of its value
  void grid(const fwi_grid& g) {
    pod(g.nz);
    pod(g.nx);
    pod(g.dx);
    pod(g.dt);
    pod(g.nt_max);
    pod(g.nsponge);
    pod(g.v_ref);
    pod(g.free_surface);
  }
};

// ---------------------------------------------------------------- validation
int check_inputs(const fwi_grid* g, const fwi_geometry* geo) {
  if (!g || !geo) return fail(FWI_ERR_ARG, "grid and geometry must not be NULL");
  if (g->nz < 1 || g->nx < 1) return fail(FWI_ERR_ARG, "nz and nx must be >= 1");
  if (g->nz > 65535) return fail(FWI_ERR_ARG, "nz must be <= 65535");
  if (!(g->dx > 0.0f) || !(g->dt > 0.0f) || !std::isfinite(g->dx) || !std::isfinite(g->dt))
    return fail(FWI_ERR_ARG, "dx and dt must be positive and finite");
  if (g->nt_max < 2) return fail(FWI_ERR_ARG, "nt_max must be >= 2");
  if (g->nsponge < kRadius) return fail(FWI_ERR_ARG, "nsponge must be >= 4");
  if (g->free_surface != 0 && g->free_surface != 1) return fail(FWI_ERR_ARG, "free_surface must be 0 or 1");
  if (!(g->v_ref > 0.0f) || !std::isfinite(g->v_ref)) return fail(FWI_ERR_ARG, "v_ref must be positive");
  const double courant = (double)g->v_ref * g->dt / g->dx;
  if (courant > FWI_CFL_LIMIT)
    return fail(FWI_ERR_CFL, "v_ref*dt/dx = " + std::to_string(courant) + " exceeds the stability bound " +
                                 std::to_string(FWI_CFL_LIMIT));
  if (geo->nshot < 0) return fail(FWI_ERR_ARG, "nshot must be >= 0");
  if (geo->nshot == 0) return FWI_OK;
  if (!geo->src_iz || !geo->src_ix || !geo->rec_ptr)
    return fail(FWI_ERR_ARG, "src_iz, src_ix and rec_ptr must not be NULL");
  if (geo->rec_ptr[0] != 0) return fail(FWI_ERR_GEOM, "rec_ptr[0] must be 0");
  for (int s = 0; s < geo->nshot; ++s) {
    if (geo->rec_ptr[s + 1] < geo->rec_ptr[s]) return fail(FWI_ERR_GEOM, "rec_ptr must be non-decreasing");
    if (geo->src_iz[s] < 0 || geo->src_iz[s] >= g->nz || geo->src_ix[s] < 0 || geo->src_ix[s] >= g->nx)
      return fail(FWI_ERR_GEOM, "source of shot " + std::to_string(s) + " lies outside the model");
    const int nt = geo->nt ? geo->nt[s] : g->nt_max;
    if (nt < 2 || nt > g->nt_max)
      return fail(FWI_ERR_GEOM, "nt of shot " + std::to_string(s) + " outside [2, nt_max]");
  }
  const int ntr = geo->rec_ptr[geo->nshot];
  if (ntr > 0 && (!geo->rec_iz || !geo->rec_ix)) return fail(FWI_ERR_ARG, "rec_iz/rec_ix must not be NULL");
  std::vector<int64_t> cells;
  for (int s = 0; s < geo->nshot; ++s) {
    cells.clear();
    for (int r = geo->rec_ptr[s]; r < geo->rec_ptr[s + 1]; ++r) {
      if (geo->rec_iz[r] < 0 || geo->rec_iz[r] >= g->nz || geo->rec_ix[r] < 0 || geo->rec_ix[r] >= g->nx)
        return fail(FWI_ERR_GEOM, "receiver " + std::to_string(r) + " lies outside the model");
      cells.push_back((int64_t)geo->rec_iz[r] * g->nx + geo->rec_ix[r]);
    }
    std::sort(cells.begin(), cells.end());
    if (std::adjacent_find(cells.begin(), cells.end()) != cells.end())
      return fail(FWI_ERR_GEOM, "shot " + std::to_string(s) + " has two receivers on one cell");
  }
  return FWI_OK;
}

// ---------------------------------------------------------------- plan
enum Phase { kPhaseFwd = 0, kPhaseRev = 1 };

struct Layout {
  size_t hdr, shots, slots, rdir, rrows, rmaps, trace_shot;
  size_t w, traces, jpart, u, lam, g, E, snap, strip, xlam, xD, xI, bu, bw, rslots, rdir2, rrows2, rmaps2, total;
};

// device header at the start of every workspace
struct Header {
  int32_t err;       // device error flag
  int32_t step;      // step counter of replayed graph chunks
  uint32_t maxbits;  // preconditioner max reduction
  int32_t pad[61];
};

struct Plan {
  uint64_t key = 0;
  uint64_t ikey = 0;  // hash of grid + geometry
  Dims d{};
  Dims dr{};  // the reverse sweep's tiling (its own rows per tile)
  int nshot = 0, ntrace = 0, max_nrec = 0, nt_max = 0;
  int S = 1, nbatch = 0, ncs = 0;
  int Sr = 1, nrbatch = 0, xcd_map_r = 0;  // reverse sweep: shots in flight, batches
  int split = 0, plain = 0, graph_steps = 0, xcd_map = 0, what = 0;
  int pf_fwd = 3, pf_rev = 1;  // prefetch distances of the forward / reverse sweeps
  int ext_h = -1, ext_T = 0;   // extended imaging: offset bound (-1: off), ring of reverse steps
  int ext_groups = 1;          // partial images (slot groups) of the extended image
  int born = 0;                // Born perturbation wavefield buffers present
  int rev_steps = 1;           // time steps per launch of the plain reverse sweep (1 or 2)
  int fwd_steps = 1;           // time steps per launch of the gradient's forward sweep (1 or 2)
  int branches = 1;            // independent chains per captured chunk of a two-step sweep
  int ulevels = kULevels, llevels = kLamLevels;
  int XT2 = 0;                 // tiles of the two-step reverse sweep along x
  double sp_a = 0.0;
  double dx = 0, dt = 0;
  std::vector<ShotDesc> shots;
  std::vector<SlotInfo> slots;  // [nbatch][S]
  std::vector<int> batch_nt;    // longest record of each batch
  // reverse batches: each forward batch's slots taken Sr at a time (same
  // checkpoint sets), longest record of each
  std::vector<SlotInfo> rslots;   // [nrbatch][Sr]
  std::vector<int> rbatch_nt;
  std::vector<int> rbatch_begin;  // [nbatch + 1]: reverse batches of forward batch b
  std::vector<RmapDir> rdir;
  std::vector<RmapRow> rrows;
  std::vector<int32_t> rmaps;
  std::vector<RmapDir> rdir2;  // receiver maps of the two-step tiling
  std::vector<RmapRow> rrows2;
  std::vector<int32_t> rmaps2;
  std::vector<int32_t> trace_shot;
  int64_t snap_stride = 0, strip_stride = 0;
  Layout L{};
  std::map<std::vector<uint64_t>, hipGraphExec_t> graphs;
  // split-mode state: workspace, v and wavelet of the last fwi_misfit_forward
  const void* fwd_ws = nullptr;
  const void* fwd_v = nullptr;
  const void* fwd_wavelet = nullptr;
  ~Plan() {
    for (auto& kv : graphs) hipGraphExecDestroy(kv.second);
  }
};

// Launch configuration: the forward sweep's shots in flight / rows per tile
// and the reverse sweep's (Sr divides S; 0 = same as the forward's), and the
// reverse sweep's time steps per launch (1 or 2).
struct ExecChoice {
  int S, TZ, graph_steps, pf_fwd, pf_rev, Sr, TZr, rsteps, fsteps;
  int branches = 0;  // independent chains per captured two-step chunk (0: kDefaultBranches)
};

std::mutex g_mutex;
std::list<std::shared_ptr<Plan>> g_plans;  // most recent first
std::map<std::vector<uint64_t>, ExecChoice> g_tuned;
hipStream_t g_capture_stream = nullptr;
std::mutex g_capture_mutex;  // graph capture (run_steps)
// further capture streams and the fork/join events of chunks captured as
// independent branches
constexpr int kMaxBranches = 4;
constexpr int kDefaultBranches = 2;
hipStream_t g_branch_stream[kMaxBranches] = {};
hipEvent_t g_fork = nullptr, g_join[kMaxBranches] = {};

int shot_nt(const fwi_grid* g, const fwi_geometry* geo, int s) { return geo->nt ? geo->nt[s] : g->nt_max; }

uint64_t inputs_hash(const fwi_grid* g, const fwi_geometry* geo) {
  Hasher h;
  h.grid(*g);
  h.pod(geo->nshot);
  if (geo->nshot > 0) {
    h.bytes(geo->src_iz, sizeof(int32_t) * geo->nshot);
    h.bytes(geo->src_ix, sizeof(int32_t) * geo->nshot);
    h.bytes(geo->rec_ptr, sizeof(int32_t) * (geo->nshot + 1));
    const int ntr = geo->rec_ptr[geo->nshot];
    if (ntr > 0) {
      h.bytes(geo->rec_iz, sizeof(int32_t) * ntr);
      h.bytes(geo->rec_ix, sizeof(int32_t) * ntr);
    }
    for (int s = 0; s < geo->nshot; ++s) h.pod(shot_nt(g, geo, s));
  }
  return h.h;
}

int default_tile_rows(int Z) {
  // long sweeps amortise the 8-row z halo; keep >= 4 tiles per column for
  // parallelism on small grids
  int tz = 64;
  while (tz > 16 && (Z + tz - 1) / tz < 4) tz /= 2;
  return tz;
}

int default_shots_in_flight(int nshot) {
  int S = std::min(nshot, 32);
  if (S >= 8) S -= S % 8;
  return std::max(S, 1);
}

// Shots per reverse launch: requested (else the forward's).  Where the reverse
// sweep follows each forward batch it takes that batch's shots a divisor at a
// time; in the autograd split (all checkpoints kept) any group size up to the
// number of shots.
int resolve_sr(int S, int req, int plain, bool split, int nshot) {
  if (plain || req <= 0) return S;
  if (split) return std::max(1, std::min(req, std::max(nshot, 1)));
  const int Sr = std::max(1, std::min(req, S));
  return S % Sr ? S : Sr;
}

void build_dims(Plan& p, const fwi_grid* g, int TZ) {
  Dims& d = p.d;
  d.nz = g->nz;
  d.nx = g->nx;
  d.N = g->nsponge;
  d.Z = d.nz + 2 * d.N;
  d.X = d.nx + 2 * d.N;
  d.off = (kWave - d.N % kWave) % kWave;
  if (d.off < kRadius) d.off += kWave;  // zero columns to the left of the grid
  d.mx0 = d.off + d.N;
  d.P = (int)align_up(d.off + d.X + kRadius, kWave);
  d.XT = d.P / kWave;
  d.TZ = TZ;
  d.fs = g->free_surface ? 1 : 0;
  d.ztop = d.fs ? d.N : 0;
  d.ZT = (d.Z - d.ztop + TZ - 1) / TZ;
  d.ring = 8 * (d.nx + d.nz);
  d.field = (int64_t)(d.Z + kGuardRows) * d.P;
  d.guard = (int64_t)kGuardRows * d.P;
  d.model = (int64_t)d.nz * d.nx;
}

// what: FWI_WS_FORWARD / GRADIENT / HESSIAN / AUTOGRAD / EXTIMAGE; ext_h: offset
// bound of the extended image (EXTIMAGE only; -1 leaves its buffers out)
std::shared_ptr<Plan> build_plan(const fwi_grid* g, const fwi_geometry* geo, const ExecChoice& ex,
                                 int plain, int what, uint64_t key, int ext_h = -1) {
  auto p = std::make_shared<Plan>();
  p->key = key;
  p->what = what;
  p->plain = plain;
  p->split = (what == FWI_WS_AUTOGRAD);
  p->nshot = geo->nshot;
  p->nt_max = g->nt_max;
  p->dx = g->dx;
  p->dt = g->dt;
  p->S = plain ? 1 : std::max(1, std::min(ex.S, std::max(geo->nshot, 1)));
  p->Sr = resolve_sr(p->S, ex.Sr, plain, p->split, geo->nshot);
  p->graph_steps = plain ? -1 : ex.graph_steps;
  p->xcd_map = (p->S >= 8 && p->S % 8 == 0) ? 1 : 0;
  p->xcd_map_r = (p->Sr >= 8 && p->Sr % 8 == 0) ? 1 : 0;
  p->pf_fwd = ex.pf_fwd;
  p->pf_rev = ex.pf_rev;
  build_dims(*p, g, ex.TZr > 0 ? ex.TZr : ex.TZ);
  p->dr = p->d;
  build_dims(*p, g, ex.TZ);
  const Dims& d = p->d;
  // two time steps per reverse launch (the plain adjoint sweep only; not with
  // a free surface)
  const bool rev2 = (what == FWI_WS_GRADIENT || what == FWI_WS_AUTOGRAD || what == FWI_WS_EXTIMAGE ||
                     what == FWI_WS_GNHVP) && !plain && !g->free_surface && ex.rsteps == 2;
  p->rev_steps = rev2 ? 2 : 1;
  // two forward steps per launch: the gradient's forward sweep (recording and
  // checkpoints), not with a free surface; two sets of (u, u, d) levels
  const bool fwd2 = (what == FWI_WS_GRADIENT || what == FWI_WS_AUTOGRAD || what == FWI_WS_EXTIMAGE) && !plain &&
                    !g->free_surface && ex.fsteps == 2;
  p->fwd_steps = fwd2 ? 2 : 1;
  p->branches = ex.branches > 0 ? ex.branches : kDefaultBranches;
  p->ulevels = fwd2 ? 2 * kULevels : (rev2 ? kULevels2 : kULevels);
  p->llevels = rev2 ? kLamLevels2 : kLamLevels;
  p->XT2 = kWavesPerBlock * ((d.X + kBlk2 - 1) / kBlk2);
  const double eta_max = 3.0 * g->v_ref * std::log(1e3) / (2.0 * d.N * g->dx);
  p->sp_a = 0.5 * g->dt * eta_max / ((double)d.N * d.N);

  const int ns = geo->nshot;
  p->ntrace = ns > 0 ? geo->rec_ptr[ns] : 0;
  p->trace_shot.assign(std::max(p->ntrace, 1), 0);
  p->shots.resize(std::max(ns, 1));
  int max_nsnap = 0;
  for (int s = 0; s < ns; ++s) {
    ShotDesc& sd = p->shots[s];
    std::memset(&sd, 0, sizeof(sd));
    sd.nt = shot_nt(g, geo, s);
    sd.K = std::max(1, (int)std::ceil(std::sqrt((double)sd.nt)));
    if (rev2) sd.K += sd.K & 1;  // two-step reverse: restarts fall on the first step of a launch
    sd.nsnap = (sd.nt - 2) / sd.K;
    max_nsnap = std::max(max_nsnap, sd.nsnap);
    sd.src_z = geo->src_iz[s] + d.N;
    sd.src_xs = geo->src_ix[s] + d.mx0;
    sd.rec_begin = geo->rec_ptr[s];
    sd.nrec = geo->rec_ptr[s + 1] - geo->rec_ptr[s];
    p->max_nrec = std::max(p->max_nrec, sd.nrec);
    sd.rdir = s * d.XT;
    sd.rdir2 = s * p->XT2;
    int zmin = g->nz, xmin = g->nx, xmax = -1;
    for (int r = sd.rec_begin; r < sd.rec_begin + sd.nrec; ++r) {
      zmin = std::min(zmin, geo->rec_iz[r]);
      xmin = std::min(xmin, geo->rec_ix[r]);
      xmax = std::max(xmax, geo->rec_ix[r]);
      p->trace_shot[r] = s;
    }
    sd.rec_z0 = sd.nrec ? zmin : 0;
    sd.xmin_m = sd.nrec ? (float)((double)xmin * g->dx) : 0.0f;
    sd.xmax_m = sd.nrec ? (float)((double)xmax * g->dx) : 0.0f;
  }
  // receiver tile maps: for each (shot, x tile) the rows holding receivers,
  // each with a 64-entry lane -> trace map
  p->rdir.assign((size_t)std::max(ns, 1) * d.XT, RmapDir{0, 0});
  for (int s = 0; s < ns; ++s) {
    std::map<std::pair<int, int>, std::vector<int>> rows;  // (xt, z) -> traces
    for (int r = geo->rec_ptr[s]; r < geo->rec_ptr[s + 1]; ++r) rows[{(geo->rec_ix[r] + d.mx0) / kWave, geo->rec_iz[r] + d.N}].push_back(r);
    for (auto& kv : rows) {
      const int xt = kv.first.first, z = kv.first.second;
      RmapDir& dir = p->rdir[(size_t)s * d.XT + xt];
      if (dir.count == 0) dir.begin = (int)p->rrows.size();
      dir.count++;
      const int map = (int)p->rmaps.size();
      p->rrows.push_back(RmapRow{z, map});
      p->rmaps.resize(map + kWave, -1);
      for (int r : kv.second) p->rmaps[map + (geo->rec_ix[r] + d.mx0) % kWave] = r;
    }
  }
  if (p->rrows.empty()) p->rrows.push_back(RmapRow{0, 0});
  if (p->rmaps.empty()) p->rmaps.assign(kWave, -1);
  // the same for the two-step tiling: wave tile t computes storage columns
  // [tile2_x0(t), +64), and the workgroups' column ranges overlap by 8, so a
  // receiver can sit in two tiles
  p->rdir2.assign((size_t)std::max(ns, 1) * std::max(p->XT2, 1), RmapDir{0, 0});
  if (rev2 || fwd2) {
    for (int s = 0; s < ns; ++s) {
      std::map<std::pair<int, int>, std::vector<int>> rows;  // (tile, z) -> traces
      for (int r = geo->rec_ptr[s]; r < geo->rec_ptr[s + 1]; ++r) {
        const int c = geo->rec_ix[r] + d.mx0;
        for (int t = 0; t < p->XT2; ++t)
          if (c >= tile2_x0(d.off, t) && c < tile2_x0(d.off, t) + kWave) rows[{t, geo->rec_iz[r] + d.N}].push_back(r);
      }
      for (auto& kv : rows) {
        const int t = kv.first.first, z = kv.first.second;
        RmapDir& dir = p->rdir2[(size_t)s * p->XT2 + t];
        if (dir.count == 0) dir.begin = (int)p->rrows2.size();
        dir.count++;
        const int map = (int)p->rmaps2.size();
        p->rrows2.push_back(RmapRow{z, map});
        p->rmaps2.resize(map + kWave, -1);
        for (int r : kv.second) p->rmaps2[map + (geo->rec_ix[r] + d.mx0 - tile2_x0(d.off, t))] = r;
      }
    }
  }
  if (p->rrows2.empty()) p->rrows2.push_back(RmapRow{0, 0});
  if (p->rmaps2.empty()) p->rmaps2.assign(kWave, -1);

  // batches: longest records first so that a batch's shots end together
  std::vector<int> order(ns);
  for (int s = 0; s < ns; ++s) order[s] = s;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return p->shots[a].nt > p->shots[b].nt; });
  p->nbatch = (ns + p->S - 1) / p->S;
  p->slots.assign((size_t)std::max(p->nbatch, 1) * p->S, SlotInfo{-1, 0});
  p->batch_nt.assign(std::max(p->nbatch, 1), 0);
  for (int i = 0; i < ns; ++i) {
    const int b = i / p->S, s = i % p->S, shot = order[i];
    p->slots[(size_t)b * p->S + s] = SlotInfo{shot, p->split ? shot : s};
    p->batch_nt[b] = std::max(p->batch_nt[b], p->shots[shot].nt);
  }
  p->ncs = p->split ? std::max(ns, 1) : p->S;
  p->rbatch_begin.assign(p->nbatch + 1, 0);
  if (p->split) {
    // every shot keeps its checkpoints until the reverse sweep, which runs
    // after all forward batches: it groups the shots (longest records first)
    // Sr at a time, independently of the forward batches
    for (int i0 = 0; i0 < ns; i0 += p->Sr) {
      int nt = 0;
      for (int k = 0; k < p->Sr; ++k) {
        const SlotInfo si = i0 + k < ns ? SlotInfo{order[i0 + k], order[i0 + k]} : SlotInfo{-1, 0};
        p->rslots.push_back(si);
        if (si.shot >= 0) nt = std::max(nt, p->shots[si.shot].nt);
      }
      p->rbatch_nt.push_back(nt);
    }
    // (a whole-gradient call would run them all after the last forward batch)
    p->rbatch_begin[p->nbatch] = (int)p->rbatch_nt.size();
  }
  for (int b = 0; b < p->nbatch && !p->split; ++b) {
    p->rbatch_begin[b] = (int)p->rbatch_nt.size();
    for (int j = 0; j < p->S; j += p->Sr) {
      int nt = 0;
      for (int k = 0; k < p->Sr; ++k) {
        const SlotInfo si = p->slots[(size_t)b * p->S + j + k];
        p->rslots.push_back(si);
        if (si.shot >= 0) nt = std::max(nt, p->shots[si.shot].nt);
      }
      if (nt == 0) {  // all idle: drop the group
        p->rslots.resize(p->rslots.size() - p->Sr);
        continue;
      }
      p->rbatch_nt.push_back(nt);
    }
  }
  if (!p->split) p->rbatch_begin[p->nbatch] = (int)p->rbatch_nt.size();
  p->nrbatch = (int)p->rbatch_nt.size();
  if (p->rslots.empty()) p->rslots.assign(p->Sr, SlotInfo{-1, 0});

  // workspace layout
  const bool grad = (what == FWI_WS_GRADIENT || what == FWI_WS_AUTOGRAD || what == FWI_WS_EXTIMAGE ||
                     what == FWI_WS_GNHVP);
  const bool hess = (what == FWI_WS_HESSIAN);
  p->born = (what == FWI_WS_BORN || what == FWI_WS_GNHVP) ? 1 : 0;
  const bool ext = (what == FWI_WS_EXTIMAGE && ext_h >= 0);
  p->ext_h = ext ? ext_h : -1;
  // the ring holds the reverse steps of one graph chunk (two per launch for
  // the two-step sweep)
  p->ext_T = ext ? (p->graph_steps > 0 ? p->graph_steps : 32) * p->rev_steps : 0;
  Layout& L = p->L;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + std::max(bytes, (size_t)4));
    return at;
  };
  L.hdr = take(sizeof(Header));
  L.shots = take(sizeof(ShotDesc) * p->shots.size());
  L.slots = take(sizeof(SlotInfo) * p->slots.size());
  L.rslots = take(sizeof(SlotInfo) * p->rslots.size());
  L.rdir = take(sizeof(RmapDir) * p->rdir.size());
  L.rrows = take(sizeof(RmapRow) * p->rrows.size());
  L.rmaps = take(sizeof(int32_t) * p->rmaps.size());
  L.rdir2 = take(sizeof(RmapDir) * p->rdir2.size());
  L.rrows2 = take(sizeof(RmapRow) * p->rrows2.size());
  L.rmaps2 = take(sizeof(int32_t) * p->rmaps2.size());
  L.trace_shot = take(sizeof(int32_t) * p->trace_shot.size());
  L.w = take(sizeof(float) * d.field);
  L.traces = take(sizeof(float) * (size_t)g->nt_max * std::max(p->ntrace, 1));
  L.jpart = take(sizeof(double) * std::max(p->ntrace, 1));
  // wavefields: guard rows in front of the first level
  L.u = take(sizeof(float) * (p->ulevels * d.field * p->ncs + d.guard));
  L.lam = grad ? take(sizeof(float) * (p->llevels * d.field * p->Sr + d.guard)) : o;
  L.g = grad ? take(sizeof(float) * d.model * p->Sr) : o;
  // E per reverse slot (gradient) or per forward slot (forward-only Hessian)
  L.E = (grad || hess) ? take(sizeof(float) * d.model * (hess ? p->S : p->Sr)) : o;
  p->snap_stride = grad ? (int64_t)max_nsnap * 2 * d.model : 0;
  p->strip_stride = grad ? (int64_t)g->nt_max * d.ring : 0;
  L.snap = grad ? take(sizeof(float) * p->snap_stride * p->ncs) : o;
  L.strip = grad ? take(sizeof(float) * p->strip_stride * p->ncs) : o;
  L.xlam = ext ? take(sizeof(float) * d.model * p->ext_T * p->Sr) : o;
  L.xD = ext ? take(sizeof(float) * d.model * p->ext_T * p->Sr) : o;
  // up to 4 slot groups fold in parallel for |h| <= 16 (one for larger offsets)
  p->ext_groups = ext ? (p->ext_h <= 16 ? std::min(p->Sr, 4) : 1) : 1;
  L.xI = ext ? take(sizeof(float) * d.model * (2 * p->ext_h + 1) * p->ext_groups) : o;
  L.bu = p->born ? take(sizeof(float) * (kULevels * d.field * p->ncs + d.guard)) : o;
  L.bw = p->born ? take(sizeof(float) * d.field) : o;
  L.total = o;
  return p;
}

template <class T>
T* at(void* ws, size_t off) { return (T*)((char*)ws + off); }

// batch: forward batch (phase kPhaseFwd) or reverse batch (kPhaseRev); two:
// the two-step reverse sweep (its own x tiling and receiver maps)
StepArgs step_args(const Plan& p, void* ws, int batch, int phase, const float* wavelet, int64_t wstride,
                   bool two = false) {
  StepArgs a{};
  const bool rev = phase == kPhaseRev;
  a.d = rev ? p.dr : p.d;
  if (two) a.d.XT = p.XT2;
  a.S = rev ? p.Sr : p.S;
  a.xcd_map = rev ? p.xcd_map_r : p.xcd_map;
  a.slots = rev ? at<SlotInfo>(ws, p.L.rslots) + (size_t)batch * p.Sr
                : at<SlotInfo>(ws, p.L.slots) + (size_t)batch * p.S;
  a.shots = at<ShotDesc>(ws, p.L.shots);
  a.rdir = at<RmapDir>(ws, two ? p.L.rdir2 : p.L.rdir);
  a.rrows = at<RmapRow>(ws, two ? p.L.rrows2 : p.L.rrows);
  a.rmaps = at<int32_t>(ws, two ? p.L.rmaps2 : p.L.rmaps);
  a.w = at<float>(ws, p.L.w);
  a.u = at<float>(ws, p.L.u) + p.d.guard;
  a.lam = at<float>(ws, p.L.lam) + p.d.guard;
  a.ustride = (int64_t)p.ulevels * p.d.field;
  a.lstride = (int64_t)p.llevels * p.d.field;
  a.g = at<float>(ws, p.L.g);
  a.E = at<float>(ws, p.L.E);
  a.traces = at<float>(ws, p.L.traces);
  a.ntrace = std::max(p.ntrace, 1);
  a.wavelet = wavelet;
  a.wstride = wstride;
  a.snap = at<float>(ws, p.L.snap);
  a.strip = at<float>(ws, p.L.strip);
  a.snap_stride = p.snap_stride;
  a.strip_stride = p.strip_stride;
  a.sp_a = p.sp_a;
  a.step_ctr = nullptr;
  a.step = 0;
  a.err = &at<Header>(ws, p.L.hdr)->err;
  a.ext_lam = p.ext_h >= 0 ? at<float>(ws, p.L.xlam) : nullptr;
  a.ext_D = p.ext_h >= 0 ? at<float>(ws, p.L.xD) : nullptr;
  a.ext_T = p.ext_T;
  a.bu = p.born ? at<float>(ws, p.L.bu) + p.d.guard : nullptr;
  a.bw = p.born ? at<float>(ws, p.L.bw) : nullptr;
  return a;
}

ExtArgs ext_args(const Plan& p, void* ws, int rbatch) {
  ExtArgs e{};
  e.d = p.d;
  e.S = p.Sr;
  e.slots = at<SlotInfo>(ws, p.L.rslots) + (size_t)rbatch * p.Sr;
  e.shots = at<ShotDesc>(ws, p.L.shots);
  e.lam = at<float>(ws, p.L.xlam);
  e.D = at<float>(ws, p.L.xD);
  e.T = p.ext_T;
  e.I = at<float>(ws, p.L.xI);
  e.hmax = p.ext_h;
  e.groups = p.ext_groups;
  e.step_ctr = nullptr;
  e.step_mul = 1;
  e.step0 = 0;
  e.count = 0;
  e.err = &at<Header>(ws, p.L.hdr)->err;
  return e;
}

hipError_t get_capture_stream(hipStream_t* out) {
  if (!g_capture_stream) {
    hipError_t e = hipStreamCreateWithFlags(&g_capture_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
  }
  *out = g_capture_stream;
  return hipSuccess;
}

// streams 1 .. n-1 for the branches of a captured chunk, and the events
hipError_t get_branch_streams(int n) {
  if (!g_fork) {
    hipError_t e = hipEventCreateWithFlags(&g_fork, hipEventDisableTiming);
    if (e != hipSuccess) return e;
  }
  for (int i = 1; i < n; ++i) {
    if (!g_branch_stream[i]) {
      hipError_t e = hipStreamCreateWithFlags(&g_branch_stream[i], hipStreamNonBlocking);
      if (e != hipSuccess) return e;
    }
    if (!g_join[i]) {
      hipError_t e = hipEventCreateWithFlags(&g_join[i], hipEventDisableTiming);
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

// slots s0 .. s0 + n - 1 of a launch as a launch of their own (the per-slot
// arrays of the reverse sweep move with them)
StepArgs slot_range(const StepArgs& a, int s0, int n) {
  StepArgs b = a;
  b.S = n;
  b.xcd_map = (n >= 8 && n % 8 == 0) ? a.xcd_map : 0;
  b.slots += s0;
  b.lam += (int64_t)s0 * a.lstride;
  b.g += (int64_t)s0 * a.d.model;
  b.E += (int64_t)s0 * a.d.model;
  if (b.ext_lam) b.ext_lam += (int64_t)s0 * a.ext_T * a.d.model;
  if (b.ext_D) b.ext_D += (int64_t)s0 * a.ext_T * a.d.model;
  return b;
}

// Run `nsteps` time steps of one phase for one batch: direct launches, or
// replays of a captured chunk of `graph_steps` launches that read the step
// base from the workspace header.
int run_steps(Plan& p, void* ws, int batch, int phase, int flags, int nsteps, const float* wavelet,
              int64_t wstride, hipStream_t stream) {
  if (nsteps <= 0) return FWI_OK;
  // the plain reverse sweep of a two-step plan, or the gradient's forward
  // sweep of one: launches of two steps each
  const bool two_rev = phase == kPhaseRev && (flags & ~kRevExt) == 0 && p.rev_steps == 2;
  const bool two_fwd = phase == kPhaseFwd && flags == (kFwdRecord | kFwdCkpt) && p.fwd_steps == 2;
  const bool two = two_rev || two_fwd;
  const int total_steps = nsteps;  // time steps (the extended image counts these)
  if (two) nsteps = (nsteps + 1) / 2;
  StepArgs a = step_args(p, ws, batch, phase, wavelet, wstride, two);
  // reverse sweeps with kRevExt keep lam and D of the last ext_T steps and
  // fold them into the extended image after every ext_T steps
  const bool ext = phase == kPhaseRev && (flags & kRevExt);
  if (ext && p.ext_h < 0) return fail(FWI_ERR_STATE, "extended image without its buffers");
  ExtArgs e = ext ? ext_args(p, ws, batch) : ExtArgs{};
  const int spl = two ? 2 : 1;  // time steps per launch
  e.step_mul = spl;
  auto launch = [&](const StepArgs& args, hipStream_t s) -> hipError_t {
    if (two_rev) return launch_reverse2(args, p.pf_rev, flags, s);
    if (two_fwd) return launch_forward2(args, p.pf_fwd == 1 ? 1 : 3, s);
    return phase == kPhaseFwd ? launch_forward(args, flags, p.pf_fwd, s)
                              : launch_reverse(args, p.pf_rev, flags, s);
  };
  const int T = p.graph_steps;
  // fold the ring after the launch that completes a window of ext_T steps,
  // or the sweep; `done` time steps so far
  auto fold_direct = [&](int k) -> hipError_t {
    const int done = std::min(spl * (k + 1), total_steps);
    if (!(done % p.ext_T == 0 || k == nsteps - 1)) return hipSuccess;
    e.step_ctr = nullptr;
    e.step0 = (done - 1) - (done - 1) % p.ext_T;
    e.count = done - e.step0;
    return launch_ext_image(e, stream);
  };
  if (T <= 0) {
    for (int k = 0; k < nsteps; ++k) {
      a.step = k;
      HIP_TRY(launch(a, stream));
      if (ext) HIP_TRY(fold_direct(k));
    }
    return FWI_OK;
  }
  if (ext && p.ext_T != T * spl) return fail(FWI_ERR_STATE, "extended-image ring differs from the graph chunk");
  int32_t* ctr = &at<Header>(ws, p.L.hdr)->step;
  // chunks of the two-step sweeps as `branches` independent chains over
  // shares of the slots, so that one chain's launches fill the others' tails
  // (the one-step sweeps' chunks stay one chain)
  const int nbr = two ? std::max(1, std::min({p.branches, a.S, kMaxBranches})) : 1;
  const std::vector<uint64_t> gkey = {(uint64_t)phase, (uint64_t)flags, (uint64_t)batch, (uint64_t)T, (uint64_t)nbr,
                                      (uint64_t)(phase == kPhaseFwd ? p.pf_fwd : p.pf_rev),
                                      (uint64_t)(uintptr_t)ws, (uint64_t)(uintptr_t)wavelet,
                                      (uint64_t)wstride, (uint64_t)ext, (uint64_t)two};
  hipGraphExec_t exec = nullptr;
  // the capture streams, the fork and join events and the plan's graph cache
  // are shared by calls from every thread
  std::unique_lock<std::mutex> capture_lock(g_capture_mutex);
  auto it = p.graphs.find(gkey);
  if (it != p.graphs.end()) {
    exec = it->second;
  } else {
    hipStream_t cs;
    HIP_TRY(get_capture_stream(&cs));
    if (nbr > 1) HIP_TRY(get_branch_streams(nbr));
    HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));
    a.step_ctr = ctr;
    hipError_t le = hipSuccess;
    if (nbr > 1) {
      // independent chains over consecutive ranges of the slots
      StepArgs ab[kMaxBranches];
      hipStream_t sb[kMaxBranches] = {cs};
      for (int i = 0; i < nbr; ++i) {
        const int s0 = a.S * i / nbr, s1 = a.S * (i + 1) / nbr;
        ab[i] = slot_range(a, s0, s1 - s0);
        if (i) sb[i] = g_branch_stream[i];
      }
      le = hipEventRecord(g_fork, cs);
      int forked = 1;  // streams that are part of the capture
      while (le == hipSuccess && forked < nbr) {
        le = hipStreamWaitEvent(sb[forked], g_fork, 0);
        if (le == hipSuccess) ++forked;
      }
      for (int k = 0; k < T && le == hipSuccess; ++k)
        for (int i = 0; i < nbr && le == hipSuccess; ++i) {
          ab[i].step = k;
          le = launch(ab[i], sb[i]);
        }
      for (int i = 1; i < forked; ++i) {
        hipError_t je = hipEventRecord(g_join[i], sb[i]);
        if (je == hipSuccess) je = hipStreamWaitEvent(cs, g_join[i], 0);
        if (le == hipSuccess) le = je;
      }
    } else {
      for (int k = 0; k < T && le == hipSuccess; ++k) {
        a.step = k;
        le = launch(a, cs);
      }
    }
    if (ext && le == hipSuccess) {
      ExtArgs ec = e;
      ec.step_ctr = ctr;
      ec.step0 = 0;
      ec.count = T * spl;
      le = launch_ext_image(ec, cs);
    }
    if (le == hipSuccess) le = launch_advance(ctr, T, cs);
    hipGraph_t graph = nullptr;
    hipError_t ee = hipStreamEndCapture(cs, &graph);
    if (le != hipSuccess) {
      if (graph) hipGraphDestroy(graph);
      return fail(FWI_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(le));
    }
    if (ee != hipSuccess) return fail(FWI_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(ee));
    hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (ie != hipSuccess) return fail(FWI_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
    p.graphs[gkey] = exec;
  }
  capture_lock.unlock();
  // whole chunks as graph replays, the remainder as direct launches, so that
  // every launch advances at least one shot
  const int full = nsteps / T;
  if (full > 0) {
    HIP_TRY(launch_set(ctr, 0, stream));
    for (int c = 0; c < full; ++c) HIP_TRY(hipGraphLaunch(exec, stream));
  }
  a.step_ctr = nullptr;
  for (int k = full * T; k < nsteps; ++k) {
    a.step = k;
    HIP_TRY(launch(a, stream));
  }
  if (ext && nsteps > full * T) {  // the remaining time steps, one window
    e.step_ctr = nullptr;
    e.step0 = full * T * spl;
    e.count = total_steps - e.step0;
    HIP_TRY(launch_ext_image(e, stream));
  }
  return FWI_OK;
}

int upload_tables(const Plan& p, void* ws, hipStream_t s) {
  HIP_TRY(hipMemcpyAsync(at<char>(ws, p.L.shots), p.shots.data(), sizeof(ShotDesc) * p.shots.size(),
                         hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(at<char>(ws, p.L.slots), p.slots.data(), sizeof(SlotInfo) * p.slots.size(),
                         hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(at<char>(ws, p.L.rslots), p.rslots.data(), sizeof(SlotInfo) * p.rslots.size(),
                         hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(at<char>(ws, p.L.rdir), p.rdir.data(), sizeof(RmapDir) * p.rdir.size(),
                         hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(at<char>(ws, p.L.rrows), p.rrows.data(), sizeof(RmapRow) * p.rrows.size(),
                         hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(at<char>(ws, p.L.rmaps), p.rmaps.data(), sizeof(int32_t) * p.rmaps.size(),
                         hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(at<char>(ws, p.L.rdir2), p.rdir2.data(), sizeof(RmapDir) * p.rdir2.size(),
                         hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(at<char>(ws, p.L.rrows2), p.rrows2.data(), sizeof(RmapRow) * p.rrows2.size(),
                         hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(at<char>(ws, p.L.rmaps2), p.rmaps2.data(), sizeof(int32_t) * p.rmaps2.size(),
                         hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(at<char>(ws, p.L.trace_shot), p.trace_shot.data(),
                         sizeof(int32_t) * p.trace_shot.size(), hipMemcpyHostToDevice, s));
  return FWI_OK;
}

// prepares the workspace for a call: tables, cleared error flag, w = dt^2 v^2/h^2
// (and the Born source factor 2 dv / v when dv is given)
int begin_call(const Plan& p, void* ws, const float* v, hipStream_t s, const float* dv = nullptr) {
  int rc = upload_tables(p, ws, s);
  if (rc) return rc;
  Header* hd = at<Header>(ws, p.L.hdr);
  HIP_TRY(launch_set(&hd->err, 0, s));
  const float vmax = (float)(FWI_CFL_LIMIT * p.dx / p.dt);  // device check in FP32
  HIP_TRY(launch_prep(p.d, v, at<float>(ws, p.L.w), p.dt, p.dx, vmax, &hd->err, s));
  if (p.born && dv) HIP_TRY(launch_prep_born(p.d, v, dv, at<float>(ws, p.L.bw), s));
  return FWI_OK;
}

int forward_batch(Plan& p, void* ws, int b, int flags, const float* wavelet, int64_t wstride,
                  hipStream_t s) {
  const SlotInfo* slots = at<SlotInfo>(ws, p.L.slots) + (size_t)b * p.S;
  HIP_TRY(launch_fill_slots(at<float>(ws, p.L.u), p.ulevels * p.d.field, p.ulevels * p.d.field + p.d.guard, slots,
                            p.S, 1, s));
  if (flags & kFwdBorn)
    HIP_TRY(launch_fill_slots(at<float>(ws, p.L.bu), kULevels * p.d.field, kULevels * p.d.field + p.d.guard, slots,
                              p.S, 1, s));
  if (int rc = run_steps(p, ws, b, kPhaseFwd, flags, p.batch_nt[b] - 1, wavelet, wstride, s)) return rc;
  if (flags == (kFwdRecord | kFwdCkpt) && p.fwd_steps == 2)
    HIP_TRY(launch_forward2_finish(at<float>(ws, p.L.u) + p.d.guard, p.ulevels * p.d.field, kULevels * p.d.field,
                                   slots, at<ShotDesc>(ws, p.L.shots), p.S, s));
  return FWI_OK;
}

int misfit_batch(Plan& p, void* ws, int b, const float* d_obs, int misfit, hipStream_t s) {
  MisfitArgs m{};
  m.slots = at<SlotInfo>(ws, p.L.slots) + (size_t)b * p.S;
  m.shots = at<ShotDesc>(ws, p.L.shots);
  m.traces = at<float>(ws, p.L.traces);
  m.dobs = d_obs;
  m.ntrace = std::max(p.ntrace, 1);
  m.nt_max = p.nt_max;
  m.kind = misfit;
  m.dt = p.dt;
  m.psi_scale = p.dx * p.dx / (p.dt * p.dt);
  m.Jpart = at<double>(ws, p.L.jpart);
  m.err = &at<Header>(ws, p.L.hdr)->err;
  HIP_TRY(launch_misfit(m, p.S, p.max_nrec, s));
  return FWI_OK;
}

// rb: reverse batch
int reverse_batch(Plan& p, void* ws, int rb, const float* wavelet, int64_t wstride, hipStream_t s,
                  int flags = 0) {
  const SlotInfo* slots = at<SlotInfo>(ws, p.L.rslots) + (size_t)rb * p.Sr;
  HIP_TRY(launch_fill_slots(at<float>(ws, p.L.lam), p.llevels * p.d.field, p.llevels * p.d.field + p.d.guard, slots,
                            p.Sr, 0, s));
  return run_steps(p, ws, rb, kPhaseRev, flags, p.rbatch_nt[rb] - 1, wavelet, wstride, s);
}

// b: reverse batch (rev, E of the reverse slots) or forward batch (E of the
// forward-only Hessian sweep)
int epilogue_batch(Plan& p, void* ws, int b, bool rev, const float* v, float* H1, float* D, int hmax,
                   int rcv_model, hipStream_t s) {
  if (!H1 && !D) return FWI_OK;
  EpiArgs e{};
  e.d = p.d;
  e.S = rev ? p.Sr : p.S;
  e.slots = rev ? at<SlotInfo>(ws, p.L.rslots) + (size_t)b * p.Sr : at<SlotInfo>(ws, p.L.slots) + (size_t)b * p.S;
  e.shots = at<ShotDesc>(ws, p.L.shots);
  e.E = at<float>(ws, p.L.E);
  e.v = v;
  e.H1 = H1;
  e.D = D;
  e.hmax = D ? hmax : 0;
  e.rcv_none = (rcv_model == FWI_RCV_NONE);
  e.h = (float)p.dx;
  e.inv_dt3 = (float)(1.0 / (p.dt * p.dt * p.dt));
  e.err = &at<Header>(ws, p.L.hdr)->err;
  HIP_TRY(launch_epilogue(e, s));
  return FWI_OK;
}

int check_outputs_hess(int hmax, int rcv_model, float* D, const fwi_grid* g) {
  if (D) {
    if (hmax < 0 || hmax > 64) return fail(FWI_ERR_ARG, "hmax must be in [0, 64]");
    if (hmax >= g->nx) return fail(FWI_ERR_ARG, "hmax must be < nx");
    if (rcv_model != FWI_RCV_PM && rcv_model != FWI_RCV_NONE) return fail(FWI_ERR_ARG, "bad rcv_model");
  }
  return FWI_OK;
}

// ---------------------------------------------------------------- autotuner
double time_steps(Plan& p, void* ws, int flags, int phase, int nsteps, const float* wavelet,
                  int64_t wstride, hipStream_t s) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return 1e30;
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    return 1e30;
  }
  double ms = 1e30;
  if (run_steps(p, ws, 0, phase, flags, 2, wavelet, wstride, s) == FWI_OK &&
      hipEventRecord(e0, s) == hipSuccess &&
      run_steps(p, ws, 0, phase, flags, nsteps, wavelet, wstride, s) == FWI_OK &&
      hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess) {
    float f = 0.0f;
    if (hipEventElapsedTime(&f, e0, e1) == hipSuccess) ms = f;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  return ms;
}

// Chooses shots in flight, rows per tile and prefetch depth of the forward
// and of the reverse sweep by timing a few launches of each candidate;
// results are cached per (grid, geometry, kind of call, GPU model).
int autotune(const fwi_grid* g, const fwi_geometry* geo, const fwi_exec* ex, int what, uint64_t ikey,
             void* ws, size_t ws_bytes, const float* v, const float* wavelet, int64_t wstride,
             hipStream_t s, ExecChoice& best) {
  const int ns = geo->nshot;
  const int Smax = best.S;
  std::vector<int> Ss, TZf, TZr, PFs, RFs;
  if (ex && ex->shots_in_flight > 0) Ss = {ex->shots_in_flight};
  else
    for (int c : {8, 16, 32, 64})
      if (c <= Smax) Ss.push_back(c);
  if (Ss.empty()) Ss = {Smax};
  // the forward sweep (one field, fewer registers) likes long tiles and many
  // shots; the reverse sweep (two fields) short tiles
  if (ex && ex->tile_rows > 0) TZf = {ex->tile_rows};
  else TZf = {16, 32, 64, 128};
  if (ex && ex->tile_rows_reverse > 0) TZr = {ex->tile_rows_reverse};
  else if (ex && ex->tile_rows > 0) TZr = {ex->tile_rows};
  else TZr = {8, 12, 16, 24, 32, 64};
  if (ex && ex->prefetch > 0) PFs = {ex->prefetch};
  else PFs = {1, 3, 7};
  if (ex && ex->prefetch_reverse > 0) RFs = {ex->prefetch_reverse};
  else RFs = {1, 3};
  std::vector<int> SRs = Ss;
  if (ex && ex->shots_in_flight_reverse > 0) SRs = {ex->shots_in_flight_reverse};
  std::vector<int> RSs;  // reverse time steps per launch
  if (ex && ex->reverse_steps > 0) RSs = {ex->reverse_steps};
  else if (g->free_surface) RSs = {1};
  else RSs = {1, 2};
  const bool grad = (what == FWI_WS_GRADIENT || what == FWI_WS_AUTOGRAD || what == FWI_WS_EXTIMAGE ||
                     what == FWI_WS_GNHVP);
  // forward time steps per launch: two for the gradient's forward sweep
  // (not the Born one), tried first so that near-ties keep the fewer bytes
  std::vector<int> FSs;
  if (ex && ex->forward_steps > 0) FSs = {ex->forward_steps};
  else if (g->free_surface || !(what == FWI_WS_GRADIENT || what == FWI_WS_AUTOGRAD || what == FWI_WS_EXTIMAGE))
    FSs = {1};
  else FSs = {2, 1};
  const int fwd_flags = grad ? (kFwdRecord | kFwdCkpt) : (what == FWI_WS_HESSIAN ? kFwdIllum : kFwdRecord);
  const int nsteps = 32;  // launches timed per candidate
  // FWI_TUNE_LOG set: each candidate's best time goes to stderr
  const bool tune_log = getenv("FWI_TUNE_LOG") != nullptr;
  // ms per time step, best of two timings of `nsteps` launches (two time
  // steps each for the two-step sweeps, so that they run as the chunk of
  // graph replays in launch chains they run as in a sweep, not as direct
  // launches), to keep the choice stable
  auto timed = [&](Plan& p, int flags, int phase) {
    const bool two = phase == kPhaseRev ? (flags == 0 && p.rev_steps == 2)
                                        : (flags == (kFwdRecord | kFwdCkpt) && p.fwd_steps == 2);
    const int n = two ? 2 * nsteps : nsteps;
    return std::min(time_steps(p, ws, flags, phase, n, wavelet, wstride, s),
                    time_steps(p, ws, flags, phase, n, wavelet, wstride, s)) / n;
  };
  struct Cand {
    int S, TZ, pf, rs, fs;
    double per_shot;  // ms per shot and time step
  };
  std::vector<Cand> F, Rv;
  std::vector<int> TZs = TZf;
  for (int t : TZr)
    if (std::find(TZs.begin(), TZs.end(), t) == TZs.end()) TZs.push_back(t);
  std::sort(TZs.begin(), TZs.end());
  for (int S : Ss) {
    for (int TZ : TZs) {
      const bool tf = std::find(TZf.begin(), TZf.end(), TZ) != TZf.end();
      const bool tr = grad && std::find(TZr.begin(), TZr.end(), TZ) != TZr.end() &&
                      std::find(SRs.begin(), SRs.end(), S) != SRs.end();
      if (!tf && !tr) continue;
      const int rs_max = *std::max_element(RSs.begin(), RSs.end());
      const double shots = std::min(S, std::max(ns, 1));
      // each candidate runs in a plan of its own layout (the two-step forward
      // sweep has twice the wavefield levels)
      auto prepare = [&](int fs) -> std::shared_ptr<Plan> {
        ExecChoice c{S, TZ, best.graph_steps, PFs[0], RFs[0], S, TZ, rs_max, fs, best.branches};
        auto p = build_plan(g, geo, c, 0, what, 0);
        if (p->L.total > ws_bytes) return nullptr;
        if (begin_call(*p, ws, v, s) != FWI_OK) return nullptr;
        if (launch_fill(at<char>(ws, p->L.u), p->L.g - p->L.u, s) != hipSuccess) return nullptr;
        return p;
      };
      // within one (S, TZ) a longer prefetch must win by 2 %, so near-ties
      // resolve to the shorter one from run to run
      double fb = 1e30;
      int fpf = PFs[0], ffs = FSs[0];
      std::shared_ptr<Plan> p;
      for (int fs : FSs) {
        p = prepare(fs);
        if (!p) continue;
        if (!tf) continue;
        for (int pf : PFs) {
          if (fs == 2 && pf == 7) continue;  // the two-step sweep prefetches 1 or 3 rows
          p->pf_fwd = pf;
          const double ms = timed(*p, fwd_flags, kPhaseFwd);
          if (ms < fb * 0.98) { fb = ms; fpf = pf; ffs = fs; }
        }
      }
      if (!p || p->fwd_steps != 1) {  // the reverse timings run in the one-step forward layout
        if (!(p = prepare(1))) continue;
      }
      if (tf && fb < 1e29) {
        F.push_back(Cand{S, TZ, fpf, 1, ffs, fb / shots});
        if (tune_log)
          fprintf(stderr, "[fwi tune] forward S %d TZ %d PF %d steps %d: %.3f us per shot-step\n", S, TZ, fpf, ffs,
                  1e3 * fb / shots);
      }
      if (tr) {
        double rb = 1e30;
        int rpf = RFs[0], rrs = RSs[0];
        for (int rs : RSs) {
          for (int pf : RFs) {
            p->rev_steps = rs;
            p->pf_rev = pf;
            const double ms = timed(*p, 0, kPhaseRev);
            if (ms < rb * 0.98) { rb = ms; rpf = pf; rrs = rs; }
          }
        }
        Rv.push_back(Cand{S, TZ, rpf, rrs, 1, rb / shots});
        if (tune_log)
          fprintf(stderr, "[fwi tune] reverse S %d TZ %d PF %d steps %d: %.3f us per shot-step\n", S, TZ, rpf, rrs,
                  1e3 * rb / shots);
      }
    }
  }
  if (F.empty()) return FWI_OK;  // nothing fitted the workspace: keep the defaults
  // near-ties (within the 2 % below) go to the reverse settings that move the
  // fewest bytes per step: two steps per launch, then more shots per launch,
  // then taller bands (fewer overlap rows read twice).
  // A short timing flatters the one-step sweep: it leaves out the slower
  // restart launches, and its small working set reuses the previous launch's
  // fields from the Infinity Cache more than over a whole sweep.
  std::stable_sort(Rv.begin(), Rv.end(), [](const Cand& x, const Cand& y) {
    if (x.rs != y.rs) return x.rs > y.rs;
    if (x.S != y.S) return x.S > y.S;
    return x.TZ > y.TZ;
  });
  // the same for the forward: two steps per launch, more shots, then longer
  // bands (fewer halo rows read twice)
  std::stable_sort(F.begin(), F.end(), [](const Cand& x, const Cand& y) {
    if (x.fs != y.fs) return x.fs > y.fs;
    if (x.S != y.S) return x.S > y.S;
    return x.TZ > y.TZ;
  });
  // per forward shots-in-flight value, the forward settings and the reverse
  // settings (shots in flight dividing the forward's; any size in the
  // autograd split), each the first of its candidates in the orders above
  // that no later one beats on its own time, by 1 % (forward) or 2 %
  // (reverse); then the shots-in-flight value whose pair is fastest, a later
  // (smaller) one having to be 2 % faster.  (The forward's margin is the
  // smaller one: at 1024 x 384 its 32-step timings put 64-row bands 2.6-3.6 %
  // behind 32-row ones, which run 4-5 % faster over a whole record.)
  double best_t = 1e300;
  ExecChoice choice = best;
  std::vector<int> fS;  // forward shots-in-flight values, in F's order
  for (const Cand& f : F)
    if (std::find(fS.begin(), fS.end(), f.S) == fS.end()) fS.push_back(f.S);
  for (int S : fS) {
    const Cand* fb = nullptr;
    for (const Cand& f : F)
      if (f.S == S && (!fb || f.per_shot < fb->per_shot * 0.99)) fb = &f;
    if (!grad) {
      if (fb->per_shot < best_t * 0.98) {
        best_t = fb->per_shot;
        choice = ExecChoice{fb->S, fb->TZ, best.graph_steps, fb->pf, best.pf_rev, fb->S, fb->TZ, 1, 1};
      }
      continue;
    }
    const Cand* rb = nullptr;
    for (const Cand& r : Rv) {
      if (what != FWI_WS_AUTOGRAD && (r.S > S || S % r.S)) continue;
      if (!rb || r.per_shot < rb->per_shot * 0.98) rb = &r;
    }
    if (!rb) continue;
    const double t = fb->per_shot + rb->per_shot;
    if (t < best_t * 0.98) {
      best_t = t;
      choice = ExecChoice{fb->S, fb->TZ, best.graph_steps, fb->pf, rb->pf, rb->S, rb->TZ, rb->rs, fb->fs};
    }
  }
  (void)ikey;
  best = choice;
  return FWI_OK;
}

// ---------------------------------------------------------------- plan lookup
struct CallCtx {
  std::shared_ptr<Plan> plan;
};

ExecChoice base_choice(const fwi_grid* g, const fwi_geometry* geo, const fwi_exec* ex) {
  ExecChoice c{};
  const int Z = g->nz + 2 * g->nsponge;
  c.S = (ex && ex->shots_in_flight > 0) ? ex->shots_in_flight : default_shots_in_flight(geo->nshot);
  c.TZ = (ex && ex->tile_rows > 0) ? ex->tile_rows : default_tile_rows(Z);
  c.graph_steps = (ex && ex->graph_steps != 0) ? ex->graph_steps : 32;
  c.pf_fwd = (ex && ex->prefetch > 0) ? ex->prefetch : 3;
  c.pf_rev = (ex && ex->prefetch_reverse > 0) ? ex->prefetch_reverse : 1;
  c.Sr = (ex && ex->shots_in_flight_reverse > 0) ? ex->shots_in_flight_reverse : 0;
  c.TZr = (ex && ex->tile_rows_reverse > 0) ? ex->tile_rows_reverse : 0;
  c.rsteps = (ex && ex->reverse_steps > 0) ? ex->reverse_steps : 1;
  c.fsteps = (ex && ex->forward_steps > 0) ? ex->forward_steps : 1;
  c.branches = (ex && ex->graph_branches > 0) ? ex->graph_branches : kDefaultBranches;
  return c;
}

std::vector<uint64_t> tune_key(const fwi_grid* g, const fwi_geometry* geo, const fwi_exec* ex, int what) {
  Hasher h;
  h.grid(*g);
  h.pod(geo->nshot);
  // extended-image and Gauss-Newton calls run the gradient's sweeps, Born
  // modelling the forward's: tune them once for each pair
  if (what == FWI_WS_EXTIMAGE || what == FWI_WS_GNHVP) what = FWI_WS_GRADIENT;
  if (what == FWI_WS_BORN) what = FWI_WS_FORWARD;
  std::vector<uint64_t> k = {h.h, (uint64_t)what, (uint64_t)(ex ? ex->shots_in_flight : 0),
                             (uint64_t)(ex ? ex->tile_rows : 0), (uint64_t)(ex ? ex->prefetch : 0),
                             (uint64_t)(ex ? ex->prefetch_reverse : 0),
                             (uint64_t)(ex ? ex->shots_in_flight_reverse : 0),
                             (uint64_t)(ex ? ex->tile_rows_reverse : 0),
                             (uint64_t)(ex ? ex->reverse_steps : 0),
                             (uint64_t)(ex ? ex->forward_steps : 0),
                             (uint64_t)(ex ? ex->graph_branches : 0)};
  int ntmax = 0, nrmax = 0;
  for (int s = 0; s < geo->nshot; ++s) {
    ntmax = std::max(ntmax, shot_nt(g, geo, s));
    nrmax = std::max(nrmax, geo->rec_ptr[s + 1] - geo->rec_ptr[s]);
  }
  k.push_back((uint64_t)ntmax);
  k.push_back((uint64_t)nrmax);
  // the tuned choice depends on the GPU model: key it by the device's arch name
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
    Hasher a;
    a.bytes(prop.gcnArchName, strnlen(prop.gcnArchName, sizeof(prop.gcnArchName)));
    a.pod(prop.multiProcessorCount);
    k.push_back(a.h);
  }
  return k;
}

// Tuned choices persist across processes in a plain text file named by the
// environment variable FWI_TUNE_CACHE: one line per key,
//   "<key words in hex> : S TZ graph_steps prefetch prefetch_reverse S_rev TZ_rev reverse_steps".
std::string key_text(const std::vector<uint64_t>& k) {
  std::string out;
  char buf[24];
  for (uint64_t w : k) {
    snprintf(buf, sizeof(buf), "%016llx ", (unsigned long long)w);
    out += buf;
  }
  return out;
}

bool cache_lookup(const std::vector<uint64_t>& k, ExecChoice& c) {
  const char* path = getenv("FWI_TUNE_CACHE");
  if (!path || !*path) return false;
  FILE* f = fopen(path, "r");
  if (!f) return false;
  const std::string want = key_text(k);
  char line[1024];
  bool found = false;
  while (fgets(line, sizeof(line), f)) {
    const char* colon = strchr(line, ':');
    if (!colon) continue;
    if (std::string(line, colon - line) != want) continue;
    ExecChoice t{};
    if (sscanf(colon + 1, "%d %d %d %d %d %d %d %d %d", &t.S, &t.TZ, &t.graph_steps, &t.pf_fwd, &t.pf_rev, &t.Sr,
               &t.TZr, &t.rsteps, &t.fsteps) == 9 &&
        (t.rsteps == 1 || t.rsteps == 2) && (t.fsteps == 1 || t.fsteps == 2) &&
        t.Sr > 0 && t.TZr >= 8 && t.TZr <= 4096 &&
        t.S > 0 && t.TZ >= 8 && t.TZ <= 4096 && (t.graph_steps == -1 || (t.graph_steps > 0 && t.graph_steps <= 1024)) &&
        (t.pf_fwd == 1 || t.pf_fwd == 3 || t.pf_fwd == 7) &&
        (t.pf_rev == 1 || t.pf_rev == 3)) {
      c = t;  // last matching line wins
      found = true;
    }
  }
  fclose(f);
  return found;
}

void cache_store(const std::vector<uint64_t>& k, const ExecChoice& c) {
  const char* path = getenv("FWI_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "%s: %d %d %d %d %d %d %d %d %d\n", key_text(k).c_str(), c.S, c.TZ, c.graph_steps, c.pf_fwd,
          c.pf_rev, c.Sr, c.TZr, c.rsteps, c.fsteps);
  fclose(f);
}

// Returns the plan for a call; with autotuning requested and no cached
// choice, runs the tuner inside `ws` first (needs a workspace sized for the
// untuned maximum, which fwi_workspace_bytes reports).
int check_exec(const fwi_exec* ex) {
  if (ex && ex->mode != FWI_EXEC_PLAIN && ex->mode != FWI_EXEC_BATCHED) return fail(FWI_ERR_ARG, "bad exec mode");
  if (ex && (ex->shots_in_flight < 0 || ex->tile_rows < 0 || ex->graph_steps < -1 ||
             ex->shots_in_flight_reverse < 0 || ex->tile_rows_reverse < 0))
    return fail(FWI_ERR_ARG, "bad exec settings");
  if (ex && ((ex->tile_rows > 0 && ex->tile_rows < 8) || (ex->tile_rows_reverse > 0 && ex->tile_rows_reverse < 8)))
    return fail(FWI_ERR_ARG, "tile_rows must be >= 8");
  if (ex && ex->prefetch != 0 && ex->prefetch != 1 && ex->prefetch != 3 && ex->prefetch != 7)
    return fail(FWI_ERR_ARG, "prefetch must be 0, 1, 3 or 7");
  if (ex && ex->prefetch_reverse != 0 && ex->prefetch_reverse != 1 && ex->prefetch_reverse != 3)
    return fail(FWI_ERR_ARG, "prefetch_reverse must be 0, 1 or 3");
  if (ex && (ex->reverse_steps < 0 || ex->reverse_steps > 2)) return fail(FWI_ERR_ARG, "reverse_steps must be 0, 1 or 2");
  if (ex && (ex->forward_steps < 0 || ex->forward_steps > 2)) return fail(FWI_ERR_ARG, "forward_steps must be 0, 1 or 2");
  if (ex && (ex->graph_branches < 0 || ex->graph_branches > kMaxBranches))
    return fail(FWI_ERR_ARG, "graph_branches must be in [0, 4]");
  return FWI_OK;
}

int get_plan(const fwi_grid* g, const fwi_geometry* geo, const fwi_exec* ex, int what, void* ws,
             size_t ws_bytes, const float* v, const float* wavelet, int64_t wstride, hipStream_t s,
             std::shared_ptr<Plan>& out, bool sizing_only, int ext_h = -1) {
  const int plain = ex && ex->mode == FWI_EXEC_PLAIN;
  if (int rc = check_exec(ex)) return rc;
  ExecChoice c = base_choice(g, geo, ex);
  const int branches = c.branches;  // not tuned: the tuner times with it
  const bool tune = !plain && ex && ex->autotune && !sizing_only;
  const uint64_t ikey = inputs_hash(g, geo);
  std::lock_guard<std::mutex> lock(g_mutex);
  if (!plain && ex && ex->autotune) {
    // the workspace is sized for the largest candidate
    if (!(ex->shots_in_flight > 0)) c.S = std::min(std::max(geo->nshot, 1), 64);
    if (!(ex->tile_rows > 0)) c.TZ = 32;
    c.Sr = 0;  // reverse buffers sized for the forward's maximum
    if (!(ex->reverse_steps > 0)) c.rsteps = 2;  // and for the two-step sweeps' levels
    if (!(ex->forward_steps > 0)) c.fsteps = 2;
  }
  if (tune) {
    const auto tk = tune_key(g, geo, ex, what);
    auto it = g_tuned.find(tk);
    ExecChoice t = c;
    if (it != g_tuned.end()) {
      c = it->second;
    } else if (cache_lookup(tk, t) && t.S <= c.S && t.Sr <= c.S) {
      g_tuned[tk] = t;
      c = t;
    } else {
      t = c;
      int rc = autotune(g, geo, ex, what, ikey, ws, ws_bytes, v, wavelet, wstride, s, t);
      if (rc) return rc;
      g_tuned[tk] = t;
      cache_store(tk, t);
      c = t;
    }
  }
  c.branches = branches;
  Hasher h;
  h.pod(ikey);
  h.pod(what == FWI_WS_AUTOGRAD ? FWI_WS_AUTOGRAD : what);
  h.pod(plain);
  h.pod(c.S);
  h.pod(c.TZ);
  h.pod(c.graph_steps);
  h.pod(c.pf_fwd);
  h.pod(c.pf_rev);
  h.pod(c.Sr);
  h.pod(c.TZr);
  h.pod(c.rsteps);
  h.pod(c.fsteps);
  h.pod(c.branches);
  h.pod(ext_h);
  const uint64_t key = h.h;
  for (auto it = g_plans.begin(); it != g_plans.end(); ++it) {
    if ((*it)->key == key) {
      out = *it;
      g_plans.splice(g_plans.begin(), g_plans, it);
      return FWI_OK;
    }
  }
  out = build_plan(g, geo, c, plain, what, key, ext_h);
  out->ikey = ikey;
  if (!sizing_only) {
    g_plans.push_front(out);
    while (g_plans.size() > 16) g_plans.pop_back();
  }
  return FWI_OK;
}

int common_checks(const fwi_grid* g, const fwi_geometry* geo, const float* v, const float* wavelet,
                  int64_t wstride, void* ws) {
  int rc = check_inputs(g, geo);
  if (rc) return rc;
  if (!v || !wavelet || !ws) return fail(FWI_ERR_ARG, "v, wavelet and workspace must not be NULL");
  if (wstride != 0 && wstride < g->nt_max) return fail(FWI_ERR_ARG, "wavelet_stride must be 0 or >= nt_max");
  return FWI_OK;
}

int ws_check(const Plan& p, size_t ws_bytes) {
  if (ws_bytes < p.L.total)
    return fail(FWI_ERR_WORKSPACE, "workspace of " + std::to_string(ws_bytes) + " bytes, need " +
                                       std::to_string(p.L.total));
  return FWI_OK;
}


// ------------------------------------------------- exact offset diagonal
// Shots are grouped by (record length, receiver set): a group's receiver term
// sum_r |G_r|^2 is one power spectrum.  Each group runs the receivers'
// impulse responses and then its shots as batches of forward sweeps that
// capture the model cells' series; the matrix-core kernel k_dft folds them
// into the spectra chunk by chunk and sums their powers per side; the offset
// sums follow.
struct DxGroup {
  int nt = 0;
  std::vector<int> shots;
  std::vector<int32_t> riz, rix;  // the receiver set (with repeats), sorted
};

struct DxLayout {
  int S = 0;              // series in flight
  size_t plan = 0;        // plan region (offset 0)
  size_t cap = 0, C = 0, PA = 0, PB = 0, W = 0, imp = 0, wav = 0, total = 0;  // W: the phase tables
  int Tn = 0, K = 0;      // largest series length and bin count
  int Tc = 0;             // time steps captured between two DFT launches (a multiple of kDftKT)
  int Cp = 0;             // columns of the DFT matrix: 2K rounded up to kDftCols
  int ntile = 0;          // cell tiles of kDftCells model cells
  int64_t R = 0;          // cells per captured row: ntile * kDftCells
};

// Run-steps held by the chunk buffer: S runs in flight capture Tc = 8192 / S
// updates (a multiple of 64) per chunk, so that fewer runs in flight buy
// longer chunks and fewer read-modify-write passes over the spectra
constexpr int kDxRunSteps = 8192;
// default runs in flight: the one-step capture sweeps of fewer runs leave
// the GPU underused (at 1024 x 384, 8 runs cost 24 ms per run against 37 ms
// with 4), more runs shorten the chunks (at 2048 x 768, 8 and 16 runs cost
// 0.5 % and 18 % more than 4): 4 on grids of at least 1.5 M padded cells,
// else 8
int dx_default_runs(const fwi_grid* g) {
  const int64_t cells = (int64_t)(g->nz + 2 * g->nsponge) * (g->nx + 2 * g->nsponge);
  return cells >= 1500000 ? 4 : 8;
}

void dx_bins(int nt, double dt, double fmax, int& L, int& K, int& nyq) {
  L = 2 * nt;
  K = L / 2 + 1;
  if (fmax > 0) K = std::min(K, (int)std::floor(fmax * L * dt + 1e-9) + 1);
  nyq = (K == L / 2 + 1);
}

std::vector<DxGroup> dx_groups(const fwi_grid* g, const fwi_geometry* geo) {
  std::map<std::pair<int, std::vector<std::pair<int, int>>>, int> index;
  std::vector<DxGroup> out;
  for (int s = 0; s < geo->nshot; ++s) {
    std::vector<std::pair<int, int>> rec;
    for (int i = geo->rec_ptr[s]; i < geo->rec_ptr[s + 1]; ++i) rec.push_back({geo->rec_iz[i], geo->rec_ix[i]});
    if (rec.empty()) continue;  // no receivers: no contribution
    std::sort(rec.begin(), rec.end());
    auto key = std::make_pair(shot_nt(g, geo, s), rec);
    auto it = index.find(key);
    if (it == index.end()) {
      DxGroup gr;
      gr.nt = key.first;
      for (auto& r : rec) {
        gr.riz.push_back(r.first);
        gr.rix.push_back(r.second);
      }
      it = index.emplace(key, (int)out.size()).first;
      out.push_back(std::move(gr));
    }
    out[it->second].shots.push_back(s);
  }
  return out;
}

// geometry of one side of a group: sources at the receivers (impulse
// responses) or the group's shots, no receivers
struct DxGeo {
  std::vector<int32_t> siz, six, ptr, nt;
  fwi_geometry g{};
  void finish() {
    ptr.assign(siz.size() + 1, 0);
    g.nshot = (int32_t)siz.size();
    g.src_iz = siz.data();
    g.src_ix = six.data();
    g.rec_ptr = ptr.data();
    g.rec_iz = ptr.data();
    g.rec_ix = ptr.data();
    g.nt = nt.data();
  }
};

DxGeo dx_side(const fwi_geometry* geo, const DxGroup& gr, bool receivers) {
  DxGeo o;
  if (receivers) {
    o.siz = gr.riz;
    o.six = gr.rix;
  } else {
    for (int s : gr.shots) {
      o.siz.push_back(geo->src_iz[s]);
      o.six.push_back(geo->src_ix[s]);
    }
  }
  o.nt.assign(o.siz.size(), gr.nt);
  o.finish();
  return o;
}

ExecChoice dx_choice(const fwi_grid* g, const fwi_exec* ex, int S) {
  const int Z = g->nz + 2 * g->nsponge;
  const int TZ = (ex && ex->tile_rows > 0) ? ex->tile_rows : default_tile_rows(Z);
  const int pf = (ex && ex->prefetch > 0) ? ex->prefetch : 1;
  // direct launches: the capture pointer is not baked into any graph
  return ExecChoice{S, TZ, 0, pf, 1, S, TZ, 1, 1};
}

int dx_layout(const fwi_grid* g, const fwi_geometry* geo, const fwi_exec* ex, int hmax, double fmax, int dft,
              DxLayout& o) {
  if (int rc = check_inputs(g, geo)) return rc;
  if (int rc = check_exec(ex)) return rc;
  if (g->free_surface) return fail(FWI_ERR_ARG, "the exact offset diagonal needs the absorbing top");
  if (hmax < 0 || hmax > 32 || hmax >= g->nx) return fail(FWI_ERR_ARG, "hmax must be in [0, 32] and < nx");
  if (!(fmax >= 0) || !std::isfinite(fmax)) return fail(FWI_ERR_ARG, "fmax must be finite and >= 0");
  if (dft != FWI_DFT_FP32 && dft != FWI_DFT_BF16X3) return fail(FWI_ERR_ARG, "dft must be FWI_DFT_FP32 or FWI_DFT_BF16X3");
  const int64_t model = (int64_t)g->nz * g->nx;
  const int Sreq = (ex && ex->shots_in_flight > 0) ? ex->shots_in_flight : dx_default_runs(g);
  o = DxLayout{};
  int Smax = 1, nshot_max = 1;
  for (const DxGroup& gr : dx_groups(g, geo)) {
    int L, K, nyq;
    dx_bins(gr.nt, g->dt, fmax, L, K, nyq);
    // a bound on the size of the spectra (K model cells per side), which a
    // band limit keeps small
    if (K > 65535) return fail(FWI_ERR_ARG, "more than 65535 frequency bins: bound the band with fmax");
    o.Tn = std::max(o.Tn, gr.nt - 1);
    o.K = std::max(o.K, K);
    nshot_max = std::max(nshot_max, (int)gr.shots.size());
    for (int side = 0; side < 2; ++side) {
      DxGeo dg = dx_side(geo, gr, side == 0);
      const int S = std::min(Sreq, std::max(dg.g.nshot, 1));
      Smax = std::max(Smax, S);
      auto p = build_plan(g, &dg.g, dx_choice(g, ex, S), 0, FWI_WS_FORWARD, 0);
      o.plan = std::max(o.plan, (size_t)p->L.total);
    }
  }
  o.S = Smax;
  const int Tn32 = (o.Tn + kDftKT - 1) / kDftKT * kDftKT;
  o.Tc = std::max(kDftKT, std::min(Tn32, std::max(64, kDxRunSteps / Smax / 64 * 64)));
  o.Cp = (2 * o.K + kDftCols - 1) / kDftCols * kDftCols;
  o.ntile = (int)((model + kDftCells - 1) / kDftCells);
  o.R = (int64_t)o.ntile * kDftCells;
  size_t off = align_up(o.plan);
  auto take = [&](size_t& field, size_t bytes) {
    field = off;
    off = align_up(off + bytes);
  };
  take(o.cap, sizeof(float) * (size_t)Smax * o.Tc * o.R);    // the chunk's series (FP32)
  take(o.C, sizeof(float) * (size_t)Smax * o.Cp * o.R);      // running spectra
  take(o.PA, sizeof(float) * (size_t)(o.Cp / 2) * o.R);      // summed powers, padded bins x cells
  take(o.PB, sizeof(float) * (size_t)(o.Cp / 2) * o.R);
  take(o.W, sizeof(float2) * (size_t)(o.Cp / 2) * (kDftKT + Tn32 / kDftKT));  // phase tables
  take(o.imp, sizeof(float) * (size_t)g->nt_max);
  take(o.wav, sizeof(float) * (size_t)nshot_max * g->nt_max);
  o.total = off;
  return FWI_OK;
}

// Scratch of fwi_gradient_static: one array per GPU, held until the process
// ends.  Host code never uses the array's name as an address: the device
// address of each GPU's copy is looked up once per device, with that device
// current, and kept.
__device__ __align__(256) unsigned char scratch[FWI_STATIC_SCRATCH_BYTES];
std::mutex g_scratch_mutex;
std::map<int, void*> g_scratch_ptr;

int static_scratch(void** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  auto it = g_scratch_ptr.find(dev);
  if (it == g_scratch_ptr.end()) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(FWI_ERR_HIP, std::string("hipGetSymbolAddress of the static scratch: ") + hipGetErrorString(e));
    it = g_scratch_ptr.emplace(dev, ptr).first;
  }
  *out = it->second;
  return FWI_OK;
}

}  // namespace
}  // namespace fwi

using namespace fwi;

// =====================================================================
// C ABI
// =====================================================================
extern "C" {

const char* fwi_last_error(void) { return g_last_error.c_str(); }

void fwi_tune_reset(void) {
  std::lock_guard<std::mutex> lock(g_mutex);
  g_tuned.clear();
}

int fwi_validate(const fwi_grid* grid, const fwi_geometry* geom) { return check_inputs(grid, geom); }

int fwi_exec_query(const fwi_grid* grid, const fwi_geometry* geom, const fwi_exec* exec, int what,
                   fwi_exec* chosen) {
  int rc = check_inputs(grid, geom);
  if (rc) return rc;
  if (!chosen) return fail(FWI_ERR_ARG, "chosen must not be NULL");
  if ((rc = check_exec(exec))) return rc;
  if (what < FWI_WS_FORWARD || what > FWI_WS_GNHVP || what == FWI_WS_PRECOND)
    return fail(FWI_ERR_ARG, "bad `what`");
  const int plain = exec && exec->mode == FWI_EXEC_PLAIN;
  ExecChoice c = base_choice(grid, geom, exec);
  if (!plain && exec && exec->autotune) {
    std::lock_guard<std::mutex> lock(g_mutex);
    const std::vector<uint64_t> tk = tune_key(grid, geom, exec, what);
    auto it = g_tuned.find(tk);
    ExecChoice t{};
    if (it != g_tuned.end()) {
      c = it->second;
    } else if (cache_lookup(tk, t) && t.S <= c.S && t.Sr <= c.S) {
      c = t;
    }
  }
  chosen->mode = exec ? exec->mode : FWI_EXEC_BATCHED;
  chosen->autotune = exec ? exec->autotune : 0;
  chosen->shots_in_flight = plain ? 1 : std::max(1, std::min(c.S, std::max(geom->nshot, 1)));
  chosen->tile_rows = c.TZ;
  chosen->graph_steps = plain ? -1 : c.graph_steps;
  chosen->prefetch = c.pf_fwd;
  chosen->prefetch_reverse = c.pf_rev;
  {
    // the reverse sweep's settings as build_plan resolves them
    chosen->shots_in_flight_reverse =
        resolve_sr(chosen->shots_in_flight, c.Sr, plain, what == FWI_WS_AUTOGRAD, geom->nshot);
    chosen->tile_rows_reverse = c.TZr > 0 ? c.TZr : c.TZ;
    chosen->reverse_steps = (plain || grid->free_surface) ? 1 : c.rsteps;
    chosen->forward_steps = (plain || grid->free_surface || what == FWI_WS_FORWARD || what == FWI_WS_HESSIAN ||
                             what == FWI_WS_BORN || what == FWI_WS_GNHVP)
                                ? 1
                                : c.fsteps;
    chosen->graph_branches = plain ? 1 : (exec && exec->graph_branches > 0 ? exec->graph_branches : kDefaultBranches);
  }
  return FWI_OK;
}

size_t fwi_workspace_bytes(const fwi_grid* grid, const fwi_geometry* geom, const fwi_exec* exec, int what,
                           int hmax) {
  if (what == FWI_WS_PRECOND) return sizeof(Header);
  if (check_inputs(grid, geom)) return 0;
  if (what < FWI_WS_FORWARD || what > FWI_WS_GNHVP) {
    fail(FWI_ERR_ARG, "bad `what`");
    return 0;
  }
  if (what == FWI_WS_EXTIMAGE && (hmax < 0 || hmax > 32 || hmax >= grid->nx)) {
    fail(FWI_ERR_ARG, "image hmax must be in [0, 32] and < nx");
    return 0;
  }
  std::shared_ptr<Plan> p;
  if (get_plan(grid, geom, exec, what, nullptr, 0, nullptr, nullptr, 0, nullptr, p, true,
               what == FWI_WS_EXTIMAGE ? hmax : -1))
    return 0;
  return p->L.total;
}

static int forward_impl(const fwi_grid* grid, const fwi_geometry* geom, const fwi_exec* exec, const float* v,
                        const float* wavelet, int64_t wavelet_stride, const float* dv, float* data,
                        void* workspace, size_t ws_bytes, hipStream_t s) {
  // dv != null: Born modelling, the recorded traces are those of the perturbation wavefield
  int rc = common_checks(grid, geom, v, wavelet, wavelet_stride, workspace);
  if (rc) return rc;
  if (!data && geom->nshot > 0 && geom->rec_ptr[geom->nshot] > 0) return fail(FWI_ERR_ARG, "data must not be NULL");
  const int what = dv ? FWI_WS_BORN : FWI_WS_FORWARD;
  std::shared_ptr<Plan> p;
  {
    std::shared_ptr<Plan> sz;
    if ((rc = get_plan(grid, geom, exec, what, nullptr, 0, nullptr, nullptr, 0, s, sz, true))) return rc;
    if ((rc = ws_check(*sz, ws_bytes))) return rc;
  }
  if ((rc = get_plan(grid, geom, exec, what, workspace, ws_bytes, v, wavelet, wavelet_stride, s, p, false)))
    return rc;
  if ((rc = ws_check(*p, ws_bytes))) return rc;
  if (geom->nshot == 0) return FWI_OK;
  if ((rc = begin_call(*p, workspace, v, s, dv))) return rc;
  for (int b = 0; b < p->nbatch; ++b)
    if ((rc = forward_batch(*p, workspace, b, kFwdRecord | (dv ? kFwdBorn : 0), wavelet, wavelet_stride, s)))
      return rc;
  HIP_TRY(launch_traces_out(at<float>(workspace, p->L.traces), p->ntrace, p->nt_max,
                            at<ShotDesc>(workspace, p->L.shots), at<int32_t>(workspace, p->L.trace_shot), data,
                            s));
  return FWI_OK;
}

int fwi_forward(const fwi_grid* grid, const fwi_geometry* geom, const fwi_exec* exec, const float* v,
                const float* wavelet, int64_t wavelet_stride, float* data, void* workspace, size_t ws_bytes,
                void* hip_stream) {
  return forward_impl(grid, geom, exec, v, wavelet, wavelet_stride, nullptr, data, workspace, ws_bytes,
                      (hipStream_t)hip_stream);
}

int fwi_misfit_value(const fwi_grid* grid, const fwi_geometry* geom, const fwi_exec* exec, const float* v,
                     const float* wavelet, int64_t wavelet_stride, const float* d_obs, int misfit, double* J,
                     void* workspace, size_t ws_bytes, void* hip_stream) {
  int rc = common_checks(grid, geom, v, wavelet, wavelet_stride, workspace);
  if (rc) return rc;
  if (misfit != FWI_MISFIT_L2 && misfit != FWI_MISFIT_TIME_INTEGRAL) return fail(FWI_ERR_ARG, "bad misfit");
  if (!J) return fail(FWI_ERR_ARG, "J must not be NULL");
  if (!d_obs && geom->nshot > 0 && geom->rec_ptr[geom->nshot] > 0) return fail(FWI_ERR_ARG, "d_obs must not be NULL");
  hipStream_t s = (hipStream_t)hip_stream;
  std::shared_ptr<Plan> p;
  {
    std::shared_ptr<Plan> sz;
    if ((rc = get_plan(grid, geom, exec, FWI_WS_FORWARD, nullptr, 0, nullptr, nullptr, 0, s, sz, true))) return rc;
    if ((rc = ws_check(*sz, ws_bytes))) return rc;
  }
  if ((rc = get_plan(grid, geom, exec, FWI_WS_FORWARD, workspace, ws_bytes, v, wavelet, wavelet_stride, s, p,
                     false)))
    return rc;
  if ((rc = ws_check(*p, ws_bytes))) return rc;
  if ((rc = begin_call(*p, workspace, v, s))) return rc;
  for (int b = 0; b < p->nbatch; ++b) {
    if ((rc = forward_batch(*p, workspace, b, kFwdRecord, wavelet, wavelet_stride, s))) return rc;
    if ((rc = misfit_batch(*p, workspace, b, d_obs, misfit, s))) return rc;
  }
  Header* hd = at<Header>(workspace, p->L.hdr);
  if (p->ntrace > 0) {
    HIP_TRY(launch_reduce_J(at<double>(workspace, p->L.jpart), p->ntrace, J, &hd->err, s));
  } else {
    HIP_TRY(launch_fill(J, sizeof(double), s));
  }
  return FWI_OK;
}

int fwi_born(const fwi_grid* grid, const fwi_geometry* geom, const fwi_exec* exec, const float* v,
             const float* wavelet, int64_t wavelet_stride, const float* dv, float* data, void* workspace,
             size_t ws_bytes, void* hip_stream) {
  if (!dv) return fail(FWI_ERR_ARG, "dv must not be NULL");
  return forward_impl(grid, geom, exec, v, wavelet, wavelet_stride, dv, data, workspace, ws_bytes,
                      (hipStream_t)hip_stream);
}

static int gradient_impl(const fwi_grid* grid, const fwi_geometry* geom, const fwi_exec* exec, const float* v,
                         const float* wavelet, int64_t wstride, const float* d_obs, int misfit, double* J,
                         const double* grad_scale, float* grad, float* illum, int hmax, int rcv_model,
                         float* offset_diag, void* ws, size_t ws_bytes, hipStream_t s, int part,
                         float* image = nullptr, int ext_h = -1, const float* dv = nullptr) {
  // dv != null (part 0 only): Gauss-Newton product, the Born data J dv act as the residual
  // part: 0 = whole gradient, 1 = forward half (split), 2 = backward half (split);
  // image != null (part 0 only): also the offset-extended image for |h| <= ext_h
  int rc = common_checks(grid, geom, v, wavelet, wstride, ws);
  if (rc) return rc;
  if ((rc = check_outputs_hess(hmax, rcv_model, offset_diag, grid))) return rc;
  const bool ext = image != nullptr;
  if (ext && (part != 0 || ext_h < 0 || ext_h > 32 || ext_h >= grid->nx))
    return fail(FWI_ERR_ARG, "image hmax must be in [0, 32] and < nx");
  if (!ext) ext_h = -1;
  const bool gn = dv != nullptr;
  if (gn && (part != 0 || ext)) return fail(FWI_ERR_ARG, "Gauss-Newton products run as one call");
  // eq. (3) taken literally is not the gradient of J: fwi_gradient only
  const bool eq3 = part != 2 && misfit == FWI_MISFIT_EQ3_LITERAL;
  if (eq3 && (part != 0 || ext || gn)) return fail(FWI_ERR_ARG, "FWI_MISFIT_EQ3_LITERAL is for fwi_gradient only");
  const int what = gn ? FWI_WS_GNHVP : ext ? FWI_WS_EXTIMAGE : (part == 0 ? FWI_WS_GRADIENT : FWI_WS_AUTOGRAD);
  if (part != 2) {
    if (misfit != FWI_MISFIT_L2 && misfit != FWI_MISFIT_TIME_INTEGRAL && !eq3) return fail(FWI_ERR_ARG, "bad misfit");
    if (!J) return fail(FWI_ERR_ARG, "J must not be NULL");
    if (!gn && !d_obs && geom->nshot > 0 && geom->rec_ptr[geom->nshot] > 0)
      return fail(FWI_ERR_ARG, "d_obs must not be NULL");
  }
  if (part != 1 && !grad && !ext) return fail(FWI_ERR_ARG, "grad must not be NULL");
  std::shared_ptr<Plan> p;
  {
    std::shared_ptr<Plan> sz;
    if ((rc = get_plan(grid, geom, exec, what, nullptr, 0, nullptr, nullptr, 0, s, sz, true, ext_h))) return rc;
    if ((rc = ws_check(*sz, ws_bytes))) return rc;
  }
  if (part == 2) {
    // the backward half must use the plan and workspace of the forward half
    std::lock_guard<std::mutex> lock(g_mutex);
    const uint64_t ikey = inputs_hash(grid, geom);
    for (auto& cand : g_plans)
      if (cand->split && cand->ikey == ikey && cand->fwd_ws == ws && cand->fwd_v == v &&
          cand->fwd_wavelet == wavelet) {
        p = cand;
        break;
      }
    if (!p) return fail(FWI_ERR_STATE, "fwi_misfit_backward without a matching fwi_misfit_forward");
  } else {
    if ((rc = get_plan(grid, geom, exec, what, ws, ws_bytes, v, wavelet, wstride, s, p, false, ext_h))) return rc;
  }
  if ((rc = ws_check(*p, ws_bytes))) return rc;
  const Plan& cp = *p;
  const size_t model_bytes = sizeof(float) * cp.d.model;
  Header* hd = at<Header>(ws, cp.L.hdr);

  if (part != 2) {
    if ((rc = begin_call(*p, ws, v, s, dv))) return rc;
    if (part == 1) {
      p->fwd_ws = nullptr;
    }
  }
  if (part != 1) {
    HIP_TRY(launch_fill(at<float>(ws, cp.L.g), model_bytes * cp.Sr, s));
    if (illum) HIP_TRY(launch_fill(illum, model_bytes, s));
    if (offset_diag) HIP_TRY(launch_fill(offset_diag, model_bytes * (2 * hmax + 1), s));
    if (ext) HIP_TRY(launch_fill(at<float>(ws, cp.L.xI), model_bytes * (2 * ext_h + 1) * cp.ext_groups, s));
  }
  for (int b = 0; b < cp.nbatch; ++b) {
    if (part != 2) {
      if ((rc = forward_batch(*p, ws, b, kFwdRecord | kFwdCkpt | (gn ? kFwdBorn : 0), wavelet, wstride, s)))
        return rc;
      if ((rc = misfit_batch(*p, ws, b, gn ? nullptr : d_obs, misfit, s))) return rc;
    }
    if (part == 0) {
      for (int rb = cp.rbatch_begin[b]; rb < cp.rbatch_begin[b + 1]; ++rb) {
        if ((rc = reverse_batch(*p, ws, rb, wavelet, wstride, s, (ext ? kRevExt : 0) | (eq3 ? kRevImgU : 0))))
          return rc;
        if ((rc = epilogue_batch(*p, ws, rb, true, v, illum, offset_diag, hmax, rcv_model, s))) return rc;
      }
    }
  }
  if (part == 2) {
    for (int rb = 0; rb < cp.nrbatch; ++rb) {
      if ((rc = reverse_batch(*p, ws, rb, wavelet, wstride, s))) return rc;
      if ((rc = epilogue_batch(*p, ws, rb, true, v, illum, offset_diag, hmax, rcv_model, s))) return rc;
    }
  }
  if (part != 2) {
    if (cp.ntrace > 0) {
      HIP_TRY(launch_reduce_J(at<double>(ws, cp.L.jpart), cp.ntrace, J, &hd->err, s));
    } else {
      HIP_TRY(launch_fill(J, sizeof(double), s));
    }
  }
  if (part != 1 && grad) {
    // eq. (3) literally: g3 = -(2/v^3) dt^2 sum lam_r[m] u[m-1]
    HIP_TRY(launch_gradient_out(cp.d, at<float>(ws, cp.L.g), cp.Sr, v, grad_scale, eq3 ? -cp.dt * cp.dt : 1.0, grad,
                                &hd->err, s));
  }
  if (ext) HIP_TRY(launch_ext_out(cp.d, at<float>(ws, cp.L.xI), cp.ext_groups, ext_h, v, image, &hd->err, s));
  if (part == 1) {
    std::lock_guard<std::mutex> lock(g_mutex);
    p->fwd_ws = ws;
    p->fwd_v = v;
    p->fwd_wavelet = wavelet;
  }
  return FWI_OK;
}

int fwi_gradient(const fwi_grid* grid, const fwi_geometry* geom, const fwi_exec* exec, const float* v,
                 const float* wavelet, int64_t wavelet_stride, const float* d_obs, int misfit, double* J,
                 float* grad, float* illum, int hmax, int rcv_model, float* offset_diag, void* workspace,
                 size_t ws_bytes, void* hip_stream) {
  return gradient_impl(grid, geom, exec, v, wavelet, wavelet_stride, d_obs, misfit, J, nullptr, grad, illum,
                       hmax, rcv_model, offset_diag, workspace, ws_bytes, (hipStream_t)hip_stream, 0);
}

int fwi_gradient_static(const fwi_grid* grid, const fwi_geometry* geom, const fwi_exec* exec, const float* v,
                        const float* wavelet, int64_t wavelet_stride, const float* d_obs, int misfit, double* J,
                        float* grad, float* illum, int hmax, int rcv_model, float* offset_diag, void* hip_stream) {
  if (int rc = check_inputs(grid, geom)) return rc;
  if (int rc = check_exec(exec)) return rc;
  if (int rc = check_outputs_hess(hmax, rcv_model, offset_diag, grid)) return rc;
  // direct launches, heuristic settings: no graph is instantiated and no
  // candidate is timed
  fwi_exec ex{};
  if (exec) ex = *exec;
  ex.graph_steps = -1;
  ex.autotune = 0;
  const size_t need = fwi_workspace_bytes(grid, geom, &ex, FWI_WS_GRADIENT, hmax);
  if (need == 0) return FWI_ERR_ARG;  // sizing failed (message set)
  if (need > FWI_STATIC_SCRATCH_BYTES)
    return fail(FWI_ERR_WORKSPACE, "fwi_gradient_static: the call needs " + std::to_string(need) +
                                       " bytes of scratch, the static array holds " +
                                       std::to_string((size_t)FWI_STATIC_SCRATCH_BYTES));
  void* ws = nullptr;
  if (int rc = static_scratch(&ws)) return rc;
  return gradient_impl(grid, geom, &ex, v, wavelet, wavelet_stride, d_obs, misfit, J, nullptr, grad, illum, hmax,
                       rcv_model, offset_diag, ws, FWI_STATIC_SCRATCH_BYTES, (hipStream_t)hip_stream, 0);
}

int fwi_extended_image(const fwi_grid* grid, const fwi_geometry* geom, const fwi_exec* exec, const float* v,
                       const float* wavelet, int64_t wavelet_stride, const float* d_obs, int misfit, double* J,
                       float* grad, int hmax, float* image, void* workspace, size_t ws_bytes, void* hip_stream) {
  if (!image) return fail(FWI_ERR_ARG, "image must not be NULL");
  return gradient_impl(grid, geom, exec, v, wavelet, wavelet_stride, d_obs, misfit, J, nullptr, grad, nullptr, 0,
                       FWI_RCV_PM, nullptr, workspace, ws_bytes, (hipStream_t)hip_stream, 0, image, hmax);
}

int fwi_gn_hvp(const fwi_grid* grid, const fwi_geometry* geom, const fwi_exec* exec, const float* v,
               const float* wavelet, int64_t wavelet_stride, const float* dv, int misfit, double* J, float* hv,
               void* workspace, size_t ws_bytes, void* hip_stream) {
  if (!dv || !hv) return fail(FWI_ERR_ARG, "dv and hv must not be NULL");
  return gradient_impl(grid, geom, exec, v, wavelet, wavelet_stride, nullptr, misfit, J, nullptr, hv, nullptr, 0,
                       FWI_RCV_PM, nullptr, workspace, ws_bytes, (hipStream_t)hip_stream, 0, nullptr, -1, dv);
}

int fwi_misfit_forward(const fwi_grid* grid, const fwi_geometry* geom, const fwi_exec* exec, const float* v,
                       const float* wavelet, int64_t wavelet_stride, const float* d_obs, int misfit, double* J,
                       void* workspace, size_t ws_bytes, void* hip_stream) {
  return gradient_impl(grid, geom, exec, v, wavelet, wavelet_stride, d_obs, misfit, J, nullptr, nullptr,
                       nullptr, 0, FWI_RCV_PM, nullptr, workspace, ws_bytes, (hipStream_t)hip_stream, 1);
}

int fwi_misfit_backward(const fwi_grid* grid, const fwi_geometry* geom, const fwi_exec* exec, const float* v,
                        const float* wavelet, int64_t wavelet_stride, const double* grad_scale, float* grad,
                        float* illum, int hmax, int rcv_model, float* offset_diag, void* workspace,
                        size_t ws_bytes, void* hip_stream) {
  return gradient_impl(grid, geom, exec, v, wavelet, wavelet_stride, nullptr, FWI_MISFIT_L2, nullptr, grad_scale,
                       grad, illum, hmax, rcv_model, offset_diag, workspace, ws_bytes, (hipStream_t)hip_stream,
                       2);
}

int fwi_hessian_diag(const fwi_grid* grid, const fwi_geometry* geom, const fwi_exec* exec, const float* v,
                     const float* wavelet, int64_t wavelet_stride, int kind, int hmax, int rcv_model, float* diag,
                     void* workspace, size_t ws_bytes, void* hip_stream) {
  int rc = common_checks(grid, geom, v, wavelet, wavelet_stride, workspace);
  if (rc) return rc;
  if (kind != FWI_HESS_EQ1 && kind != FWI_HESS_OFFSET) return fail(FWI_ERR_ARG, "bad kind");
  if (!diag) return fail(FWI_ERR_ARG, "diag must not be NULL");
  float* H1 = kind == FWI_HESS_EQ1 ? diag : nullptr;
  float* D = kind == FWI_HESS_OFFSET ? diag : nullptr;
  if ((rc = check_outputs_hess(hmax, rcv_model, D, grid))) return rc;
  hipStream_t s = (hipStream_t)hip_stream;
  std::shared_ptr<Plan> p;
  {
    std::shared_ptr<Plan> sz;
    if ((rc = get_plan(grid, geom, exec, FWI_WS_HESSIAN, nullptr, 0, nullptr, nullptr, 0, s, sz, true))) return rc;
    if ((rc = ws_check(*sz, ws_bytes))) return rc;
  }
  if ((rc = get_plan(grid, geom, exec, FWI_WS_HESSIAN, workspace, ws_bytes, v, wavelet, wavelet_stride, s, p,
                     false)))
    return rc;
  if ((rc = ws_check(*p, ws_bytes))) return rc;
  const size_t model_bytes = sizeof(float) * p->d.model;
  HIP_TRY(launch_fill(diag, model_bytes * (D ? (2 * hmax + 1) : 1), s));
  if (geom->nshot == 0) return FWI_OK;
  if ((rc = begin_call(*p, workspace, v, s))) return rc;
  for (int b = 0; b < p->nbatch; ++b) {
    if ((rc = forward_batch(*p, workspace, b, kFwdIllum, wavelet, wavelet_stride, s))) return rc;
    if ((rc = epilogue_batch(*p, workspace, b, false, v, H1, D, hmax, rcv_model, s))) return rc;
  }
  return FWI_OK;
}

size_t fwi_offset_diag_exact_workspace_bytes(const fwi_grid* grid, const fwi_geometry* geom, const fwi_exec* exec,
                                             int hmax, double fmax, int dft) {
  DxLayout o;
  if (dx_layout(grid, geom, exec, hmax, fmax, dft, o)) return 0;
  return o.total;
}

int fwi_offset_diag_exact(const fwi_grid* grid, const fwi_geometry* geom, const fwi_exec* exec, const float* v,
                          const float* wavelet, int64_t wavelet_stride, int hmax, double fmax, int dft, float* diag,
                          void* workspace, size_t ws_bytes, void* hip_stream) {
  int rc = common_checks(grid, geom, v, wavelet, wavelet_stride, workspace);
  if (rc) return rc;
  if (!diag) return fail(FWI_ERR_ARG, "diag must not be NULL");
  DxLayout o;
  if ((rc = dx_layout(grid, geom, exec, hmax, fmax, dft, o))) return rc;
  if (ws_bytes < o.total)
    return fail(FWI_ERR_WORKSPACE, "workspace of " + std::to_string(ws_bytes) + " bytes, need " +
                                       std::to_string(o.total));
  hipStream_t s = (hipStream_t)hip_stream;
  const int nz = grid->nz, nx = grid->nx;
  const int64_t model = (int64_t)nz * nx;
  const int split = dft == FWI_DFT_BF16X3;
  HIP_TRY(launch_fill(diag, sizeof(float) * model * (2 * hmax + 1), s));
  const std::vector<DxGroup> groups = dx_groups(grid, geom);
  if (groups.empty()) return FWI_OK;
  float* cap = at<float>(workspace, o.cap);
  float* C = at<float>(workspace, o.C);
  float* PA = at<float>(workspace, o.PA);
  float* PB = at<float>(workspace, o.PB);
  float2* Tb = at<float2>(workspace, o.W);
  float* imp = at<float>(workspace, o.imp);
  float* wav = at<float>(workspace, o.wav);
  // the impulse [1, 0, 0, ...] that starts a receiver's response
  HIP_TRY(launch_fill(imp, sizeof(float) * grid->nt_max, s));
  HIP_TRY(launch_set((int32_t*)imp, 0x3f800000, s));
  const int Sreq = (exec && exec->shots_in_flight > 0) ? exec->shots_in_flight : dx_default_runs(grid);
  for (const DxGroup& gr : groups) {
    const int Tn = gr.nt - 1;
    int L, K, nyq;
    dx_bins(gr.nt, grid->dt, fmax, L, K, nyq);
    const int nslab_all = (Tn + kDftKT - 1) / kDftKT;
    const int Cp = (2 * K + kDftCols - 1) / kDftCols * kDftCols;
    float2* Ph = Tb + (size_t)(Cp / 2) * kDftKT;
    HIP_TRY(launch_dft_tables(Tb, Ph, nslab_all, Cp / 2, K, L, s));
    HIP_TRY(launch_fill(PA, sizeof(float) * (size_t)(Cp / 2) * o.R, s));
    HIP_TRY(launch_fill(PB, sizeof(float) * (size_t)(Cp / 2) * o.R, s));
    // the group's shots' wavelets, gathered in group order
    const float* wsrc = wavelet;
    int64_t wst = 0;
    if (wavelet_stride != 0) {
      for (size_t i = 0; i < gr.shots.size(); ++i)
        HIP_TRY(hipMemcpyAsync(wav + i * (size_t)grid->nt_max, wavelet + (int64_t)gr.shots[i] * wavelet_stride,
                               sizeof(float) * gr.nt, hipMemcpyDeviceToDevice, s));
      wsrc = wav;
      wst = grid->nt_max;
    }
    const int32_t* err = nullptr;  // the last plan's error flag (set if v fails its check)
    for (int side = 0; side < 2; ++side) {
      const bool rcv = side == 0;
      DxGeo dg = dx_side(geom, gr, rcv);
      const int S = std::min(Sreq, std::max(dg.g.nshot, 1));
      auto p = build_plan(grid, &dg.g, dx_choice(grid, exec, S), 0, FWI_WS_FORWARD, 0);
      if (p->L.total > o.plan || p->S > o.S) return fail(FWI_ERR_STATE, "exact offset diagonal: plan outgrew its region");
      if ((rc = begin_call(*p, workspace, v, s))) return rc;
      err = &at<Header>(workspace, p->L.hdr)->err;
      const int flags = rcv ? kFwdCapU : kFwdCapD;
      for (int b = 0; b < p->nbatch; ++b) {
        int nact = 0;
        for (int i = 0; i < p->S; ++i) nact += p->slots[(size_t)b * p->S + i].shot >= 0;
        const SlotInfo* slots = at<SlotInfo>(workspace, p->L.slots) + (size_t)b * p->S;
        HIP_TRY(launch_fill_slots(at<float>(workspace, p->L.u), p->ulevels * p->d.field,
                                  p->ulevels * p->d.field + p->d.guard, slots, p->S, 1, s));
        StepArgs a = step_args(*p, workspace, b, kPhaseFwd, rcv ? imp : wsrc, rcv ? 0 : wst, false);
        a.cap = cap;
        a.cap_T = o.Tc;
        a.cap_R = o.R;
        // the series in chunks of Tc updates, each folded into the spectra by
        // the matrix cores; the run's last chunk adds the powers to its side
        for (int k0 = 0; k0 < Tn; k0 += o.Tc) {
          const int tc = std::min(o.Tc, Tn - k0);
          a.cap_n0 = k0;
          for (int k = k0; k < k0 + tc; ++k) {
            a.step = k;
            HIP_TRY(launch_forward(a, flags, p->pf_fwd, s));
          }
          DftArgs da{};
          da.X = cap;
          da.R = o.R;
          da.xslot = (int64_t)o.Tc * o.R;
          da.tc = tc;
          da.nslab = (tc + kDftKT - 1) / kDftKT;
          da.Tb = Tb;
          da.Ph = Ph;
          da.Kp = Cp / 2;
          da.j0 = k0 / kDftKT;
          da.Cp = Cp;
          da.C = C;
          da.first = k0 == 0;
          da.last = k0 + tc >= Tn;
          da.P = rcv ? PB : PA;
          da.K = K;
          da.model = model;
          da.nslots = nact;
          da.ntile = o.ntile;
          HIP_TRY(launch_dft(da, split, s));
        }
      }
    }
    // (4 / v^6) h^4 / (dt^4 L): the source series is D / dt^2, the receiver
    // series h^2 u (the impulse enters as 1 / h^2)
    const double h2 = grid->dx * grid->dx, dt2 = grid->dt * grid->dt;
    const float scale = (float)(4.0 * h2 * h2 / (dt2 * dt2 * L));
    HIP_TRY(launch_diag_products(PA, PB, o.R, K, nyq, nz, nx, hmax, v, scale, diag, err, s));
  }
  return FWI_OK;
}

int fwi_precondition(const fwi_grid* grid, const float* v, const float* grad, int kind, const float* hdiag,
                     int hmax, float eps, float* out, void* workspace, size_t ws_bytes, void* hip_stream) {
  if (!grid || !v || !grad || !hdiag || !out || !workspace) return fail(FWI_ERR_ARG, "NULL argument");
  if (grid->nz < 1 || grid->nx < 1) return fail(FWI_ERR_ARG, "nz and nx must be >= 1");
  if (kind != FWI_PRECOND_SHOT && kind != FWI_PRECOND_OFFSET) return fail(FWI_ERR_ARG, "bad kind");
  if (kind == FWI_PRECOND_OFFSET && (hmax < 0 || hmax > 64)) return fail(FWI_ERR_ARG, "hmax must be in [0, 64]");
  if (!(eps >= 0.0f) || !std::isfinite(eps)) return fail(FWI_ERR_ARG, "eps must be >= 0");
  if (ws_bytes < sizeof(Header)) return fail(FWI_ERR_WORKSPACE, "precondition workspace too small");
  Header* hd = (Header*)workspace;
  HIP_TRY(launch_precond(grid->nz, grid->nx, v, grad, kind, hdiag, kind == FWI_PRECOND_OFFSET ? hmax : 0, eps,
                         out, &hd->maxbits, (hipStream_t)hip_stream));
  return FWI_OK;
}

int fwi_status(const void* workspace, void* hip_stream) {
  if (!workspace) return fail(FWI_ERR_ARG, "workspace must not be NULL");
  int32_t err = 0;
  HIP_TRY(hipMemcpyAsync(&err, workspace, sizeof(int32_t), hipMemcpyDeviceToHost, (hipStream_t)hip_stream));
  HIP_TRY(hipStreamSynchronize((hipStream_t)hip_stream));
  if (err) return fail(FWI_ERR_NONFINITE, "velocity non-finite, non-positive or above the CFL bound");
  return FWI_OK;
}

}  // extern "C"
