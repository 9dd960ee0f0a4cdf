// fvm_api.hip -- the C ABI (include/fvm.h): argument checking, plans, the
// ping-pong schedule, HIP-graph replay of step sequences, status handling.
// Host code only; the kernels live in fvm_kernels.hip, fvm_batch.hip and
// fvm_adjoint.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <cstdio>
#include <fstream>
#include <list>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/fvm.h"
#include "fvm_host.hpp"
#include "fvm_internal.hpp"

namespace fvm {
void* step_kernel_ptr(int model, int bc, int wpb, int cpl, bool halo);
hipError_t launch_resident_run(const StepArgs& a, int model, double* w_last, double* w_prev,
                               int nsteps, hipStream_t st);
hipError_t launch_step(const StepArgs& a, int model, hipStream_t st);
hipError_t launch_cfl(const CflArgs& a, int model, hipStream_t st);
hipError_t launch_clear_scratch(GridScratch* s, int n, hipStream_t st);
hipError_t launch_set_log(GridScratch* s, int n, double* base, int cap, int stride,
                          hipStream_t st);
hipError_t launch_adjoint(const AdjointArgs& a, int model, const double* ug, hipStream_t st);
hipError_t launch_spray_adjoint(const AdjointArgs& a, const double* ug, hipStream_t st,
                                bool src);
hipError_t launch_maxent_adjoint_source(const AdjointArgs& a, const double* ug, hipStream_t st);

GridGeom grid_geometry(const fvm_params& p) {
  GridGeom g{};
  g.nx = p.nx;
  g.ny = p.ny;
  g.bc = p.bc;
  if (p.layout == FVM_LAYOUT_ROWS) {
    g.ld = fvm_nvar(p.model) * p.ld;
    g.plane = static_cast<size_t>(p.ld);
    g.uld = 2 * p.ld;
    g.uplane = static_cast<size_t>(p.ld);
  } else {
    g.ld = p.ld;
    g.plane = static_cast<size_t>(p.ld) * p.ny;
    g.uld = p.ld;
    g.uplane = g.plane;
  }
  g.rld = p.ld;
  g.dx = p.lx / p.nx;
  g.dy = p.ly / p.ny;
  g.cfl = p.cfl;
  g.dt_max = p.dt_max;
  g.hmin = g.dx < g.dy ? g.dx : g.dy;
  return g;
}

}  // namespace fvm

using namespace fvm;

namespace {

constexpr int kDefaultRows = 64;
constexpr int kDefaultWpb = 4;
// Runs are cut into graphs of 32, 16, 8, 4, 2 and 1 steps; the first run of
// a kind builds every chunk from both ping-pong buffers, so later runs of any
// length only replay cached graphs (no graph is built between the caller's
// launches).
constexpr int kGraphChunk = 32;
constexpr int kChunkSizes[6] = {32, 16, 8, 4, 2, 1};
constexpr size_t kGraphCacheMax = 40;

bool valid_params(const fvm_params* p) {
  if (!p) return false;
  if (fvm_nvar(p->model) == 0) return false;
  if (p->bc != FVM_PERIODIC && p->bc != FVM_TRANSMISSIVE && p->bc != FVM_DIRICHLET)
    return false;
  if (p->nx < 1 || p->ny < 1 || p->npart_x < 1 || p->npart_y < 1) return false;
  if (p->nx % p->npart_x != 0 || p->ny % p->npart_y != 0) return false;
  if (p->ld < p->nx) return false;
  if (p->layout != FVM_LAYOUT_PLANES && p->layout != FVM_LAYOUT_ROWS) return false;
  if (static_cast<long long>(p->ld) * fvm_nvar(p->model) > 2147483647ll) return false;
  if (!(p->lx > 0) || !(p->ly > 0) || !std::isfinite(p->lx) || !std::isfinite(p->ly)) return false;
  if (!(p->cfl > 0) || !std::isfinite(p->cfl)) return false;
  if (!(p->dt_max >= 0) || !std::isfinite(p->dt_max)) return false;
  const double cells = static_cast<double>(p->ld) * p->ny * fvm_nvar(p->model);
  if (cells > 9.0e15) return false;
  if (p->model == FVM_EULER && !(p->gamma > 1.0 && std::isfinite(p->gamma))) return false;
  if (p->model == FVM_ADV && !(std::isfinite(p->ax) && std::isfinite(p->ay))) return false;
  if (p->model == FVM_SPRAY) {
    if (!(p->K >= 0) || !std::isfinite(p->K)) return false;
    if (!(p->theta > 0)) return false;
    if (!(p->s_eps > 0 && p->s_eps < 1)) return false;
  }
  if (p->closure != FVM_CLOSURE_LOGNORMAL && p->closure != FVM_CLOSURE_MAXENT) return false;
  if (p->closure == FVM_CLOSURE_MAXENT && p->model != FVM_SPRAY) return false;
  return true;
}

// The kernel family of a grid: the model, or the transport-then-source pair
// of the spray with the entropy-maximising closure.
static int kernel_model(const fvm_params& p) {
  return p.model == FVM_SPRAY && p.closure == FVM_CLOSURE_MAXENT ? kSprayMaxEnt : p.model;
}

ModelConsts model_consts(const fvm_params& p) {
  ModelConsts m{};
  m.gamma = p.gamma;
  m.gm1 = p.gamma - 1.0;
  m.ax = p.ax;
  m.ay = p.ay;
  m.K = p.K;
  m.inv_theta = std::isinf(p.theta) ? 0.0 : 1.0 / p.theta;
  m.s_eps = p.s_eps;
  m.log_s_eps = p.s_eps > 0 ? std::log(p.s_eps) : 0.0;
  return m;
}


Tiling tiling(const GridGeom& g, int rows, int wpb, int cpl) {
  Tiling t{};
  t.rows = rows;
  t.wpb = wpb;
  t.cpl = cpl;
  const int w = strip_width(cpl) * wpb;
  t.tiles_x = (g.nx + w - 1) / w;
  t.tiles_y = (g.ny + rows - 1) / rows;
  t.ntiles = t.tiles_x * t.tiles_y;
  return t;
}

// The adjoint kernel's strips: 128 columns with two cells per lane, or 62
// columns with one (lanes 0 and 63 only supply the halo).
Tiling adjoint_tiling(const GridGeom& g, int rows, int wpb, int cpl) {
  Tiling t = tiling(g, rows, wpb, cpl);
  if (cpl == 1) {
    const int w = kOutPerWave * wpb;
    t.tiles_x = (g.nx + w - 1) / w;
    t.ntiles = t.tiles_x * t.tiles_y;
  }
  return t;
}

// Default tile shape for a grid: the widest workgroup (up to 8 strips) the
// grid's width fills, and the tallest strips (up to 64 rows) that still give
// about 2048 wave strips, i.e. two per SIMD on 256 CUs. On the 4096^2 Euler
// grid this is the measured optimum (64 rows, 8 strips); smaller grids get
// shorter strips instead of idle CUs. fvm_autotune refines it by measurement.
void default_tiling(const fvm_params& p, int cpl, int* rows, int* wpb) {
  // the spray step holds more registers per lane (fewer waves fit), the
  // advection step far fewer
  const long long target = p.model == FVM_SPRAY ? 1024 : (p.model == FVM_ADV ? 4096 : 2048);
  const int wmax = p.model == FVM_SPRAY ? 4 : 8;
  const int width = strip_width(cpl);
  const long long strips_x = (p.nx + width - 1) / width;
  int w = 1;
  while (w < wmax && 2 * w <= strips_x) w *= 2;
  long long r = strips_x * p.ny / target;
  r = r < 4 ? 4 : (r > 64 ? 64 : r);
  *rows = static_cast<int>(r);
  *wpb = w;
}

bool valid_tiling(int rows, int wpb) {
  return rows >= 1 && rows <= 4096 && (wpb == 1 || wpb == 2 || wpb == 4 || wpb == 8);
}

int dev_err(hipError_t e) { return e == hipSuccess ? FVM_OK : FVM_EDEVICE; }

int status_from_bits(unsigned int st) {
  if (st & kStatusNonFinite) return FVM_ENONFINITE;
  if (st & kStatusCfl) return FVM_ECFL;
  if (st & kStatusDt) return FVM_EINVAL;
  return FVM_OK;
}

struct GraphKey {
  int kind;              // 0 adaptive run, 1 dts run, 2 tuner's dry run, 3 fixed-dt run
  int nsteps;
  const double* start;   // input buffer of the first step
  const double* other;
  const double* dts;
  int k0;
  int rows, wpb, cpl;
  double dt;             // kind 3
  const double* me_lam;  // entropy closure: the multiplier buffer, and whether
  bool me_warm;          // the graph's first step starts from it
  bool operator==(const GraphKey& o) const {
    return kind == o.kind && nsteps == o.nsteps && start == o.start && other == o.other &&
           dts == o.dts && k0 == o.k0 && rows == o.rows && wpb == o.wpb &&
           cpl == o.cpl && dt == o.dt && me_lam == o.me_lam && me_warm == o.me_warm;
  }
};

struct CachedGraph {
  GraphKey key;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

}  // namespace

struct fvm_grid {
  fvm_params p{};
  int nv = 0;
  GridGeom g{};
  ModelConsts m{};
  int rows = kDefaultRows, wpb = kDefaultWpb;
  int adj_rows = kDefaultRows, adj_wpb = kDefaultWpb;  // adjoint kernel tile shape
  int adj_cpl = 1;   // adjoint cells per lane (the tuner may pick 2 where allowed)
  int cpl_req = 0;   // requested cells per lane (0: the widest the buffers allow)
  bool resident = true;  // small grids run whole adaptive runs in one workgroup
  int cpl = 1;       // layout in use
  double* w_a = nullptr;
  double* w_b = nullptr;
  double* cur = nullptr;
  const double* ug = nullptr;
  double ghost[4 * kMaxVar] = {};  // Dirichlet states, ghost[side * kMaxVar + v]
  Halo halo{};                     // rows from the caller's buffers
  double* me_lam = nullptr;        // entropy closure: the caller's multiplier buffer
  bool me_valid = false;           // it holds the multipliers of the current state's cells
  GridScratch* scr = nullptr;
  const double* log_armed = nullptr;  // dt log the scratch currently points to
  hipStream_t stream = nullptr;
  bool bound = false;
  bool speeds_valid = false;
  std::list<CachedGraph> graphs;

  ~fvm_grid() { clear_graphs(); }
  void clear_graphs() {
    for (auto& c : graphs) {
      if (c.exec) (void)hipGraphExecDestroy(c.exec);
      if (c.graph) (void)hipGraphDestroy(c.graph);
    }
    graphs.clear();
  }
  double* other(const double* w) const { return w == w_a ? w_b : w_a; }

  // doubles in one state (either layout)
  size_t elems() const { return static_cast<size_t>(nv) * p.ny * p.ld; }

  StepArgs step_args(const double* win, double* wout, int mode) const {
    StepArgs a{};
    a.win = win;
    a.wout = wout;
    a.ug = ug;
    a.scr = scr;
    a.mode = mode;
    a.g = g;
    a.t = tiling(g, rows, wpb, cpl);
    a.m = m;
    for (int k = 0; k < 4 * kMaxVar; ++k) a.ghost[k] = ghost[k];
    a.halo = halo;
    return a;
  }
};

extern "C" {

const char* fvm_strerror(int status) {
  switch (status) {
    case FVM_OK: return "ok";
    case FVM_EINVAL: return "invalid argument";
    case FVM_EDEVICE: return "HIP runtime error";
    case FVM_ECFL: return "fixed time step violates the CFL condition";
    case FVM_ENONFINITE: return "non-finite or non-physical state";
    case FVM_EUNSUPPORTED: return "operation not supported for this model";
    case FVM_EIO: return "file output failed";
    default: return "unknown status";
  }
}

int fvm_nvar(int model) {
  switch (model) {
    case FVM_ADV: return 1;
    case FVM_EULER: return 4;
    case FVM_SPRAY: return 6;
    default: return 0;
  }
}

int fvm_validate(const fvm_params* p) { return valid_params(p) ? FVM_OK : FVM_EINVAL; }

size_t fvm_scratch_bytes(const fvm_params* p) {
  if (!valid_params(p)) return 0;
  return sizeof(GridScratch);
}

int fvm_create(const fvm_params* p, fvm_grid** out) {
  if (!out) return FVM_EINVAL;
  *out = nullptr;
  if (!valid_params(p)) return FVM_EINVAL;
  if (p->closure == FVM_CLOSURE_MAXENT && p->bc == FVM_DIRICHLET) return FVM_EUNSUPPORTED;
  fvm_grid* g = new (std::nothrow) fvm_grid();
  if (!g) return FVM_EINVAL;
  g->p = *p;
  g->nv = fvm_nvar(p->model);
  default_tiling(*p, 2, &g->rows, &g->wpb);
  default_tiling(*p, 1, &g->adj_rows, &g->adj_wpb);
  g->g = grid_geometry(*p);
  g->m = model_consts(*p);
  *out = g;
  return FVM_OK;
}

int fvm_destroy(fvm_grid* g) {
  delete g;
  return FVM_OK;
}

// Two cells per lane needs an even pitch and 16-byte aligned buffers.
static bool wide_layout_ok(const fvm_grid* g) {
  auto al = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
  return g->p.ld % 2 == 0 && al(g->w_a) && al(g->w_b) && (!g->ug || al(g->ug));
}

// The adjoint covers every model and closure, without halo rows.
static bool adjoint_supported(const fvm_grid* g) { return !g->halo.s && !g->halo.n; }

// The adjoint's lane layout for one launch: two cells per lane needs an even
// pitch and 16-byte aligned state and multiplier buffers.
static int adjoint_cpl(const fvm_grid* g, const double* w, const double* li, const double* lo) {
  auto al = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
  return g->adj_cpl == 2 && g->p.ld % 2 == 0 && al(w) && al(li) && al(lo) ? 2 : 1;
}

static void choose_layout(fvm_grid* g) {
  const int want = g->cpl_req ? g->cpl_req : 2;
  const int cpl = (want == 2 && g->bound && wide_layout_ok(g)) ? 2 : 1;
  if (cpl != g->cpl) g->clear_graphs();
  g->cpl = cpl;
}

int fvm_bind(fvm_grid* g, double* w_a, double* w_b, const double* ug, void* scratch,
             void* stream) {
  if (!g || !w_a || !w_b || !scratch || w_a == w_b) return FVM_EINVAL;
  if ((reinterpret_cast<uintptr_t>(scratch) & 255) != 0) return FVM_EINVAL;
  if ((reinterpret_cast<uintptr_t>(w_a) & 7) || (reinterpret_cast<uintptr_t>(w_b) & 7))
    return FVM_EINVAL;
  if (g->p.model == FVM_SPRAY && !ug) return FVM_EINVAL;
  if (g->p.model != FVM_SPRAY && ug) return FVM_EINVAL;
  g->clear_graphs();
  g->w_a = w_a;
  g->w_b = w_b;
  g->cur = w_a;
  g->ug = ug;
  g->scr = static_cast<GridScratch*>(scratch);
  g->stream = static_cast<hipStream_t>(stream);
  g->bound = true;
  choose_layout(g);
  g->speeds_valid = false;
  g->me_valid = false;
  g->log_armed = nullptr;
  return dev_err(launch_clear_scratch(g->scr, 1, g->stream));
}

int fvm_set_boundary_states(fvm_grid* g, const double* ghost) {
  if (!g || !ghost || g->p.bc != FVM_DIRICHLET) return FVM_EINVAL;
  for (int k = 0; k < 4 * g->nv; ++k)
    if (!std::isfinite(ghost[k])) return FVM_EINVAL;
  for (int side = 0; side < 4; ++side)
    for (int v = 0; v < g->nv; ++v) g->ghost[side * kMaxVar + v] = ghost[side * g->nv + v];
  g->clear_graphs();  // the cached graphs hold the previous states
  return FVM_OK;
}

int fvm_set_halo_rows(fvm_grid* g, const double* south, const double* north) {
  if (!g) return FVM_EINVAL;
  if ((g->p.bc == FVM_DIRICHLET || g->p.closure == FVM_CLOSURE_MAXENT) && (south || north))
    return FVM_EUNSUPPORTED;
  g->halo.s = south;
  g->halo.n = north;
  g->clear_graphs();  // the cached graphs hold the previous pointers
  return FVM_OK;
}

int fvm_set_closure_buffer(fvm_grid* g, double* lam) {
  if (!g) return FVM_EINVAL;
  if (g->p.closure != FVM_CLOSURE_MAXENT) return lam ? FVM_EUNSUPPORTED : FVM_OK;
  if (lam && (reinterpret_cast<uintptr_t>(lam) & 7)) return FVM_EINVAL;
  g->me_lam = lam;
  g->me_valid = false;
  g->clear_graphs();  // the cached graphs hold the previous pointer
  return FVM_OK;
}

int fvm_set_stream(fvm_grid* g, void* stream) {
  if (!g) return FVM_EINVAL;
  g->stream = static_cast<hipStream_t>(stream);
  return FVM_OK;
}

int fvm_current(const fvm_grid* g, double** w) {
  if (!g || !w || !g->bound) return FVM_EINVAL;
  *w = g->cur;
  return FVM_OK;
}

}  // extern "C"

namespace fvm {
int grid_view(const fvm_grid* g, GridView* v) {
  if (!g || !v || !g->bound) return FVM_EINVAL;
  v->p = g->p;
  v->g = g->g;
  v->nv = g->nv;
  v->cur = g->cur;
  v->stream = g->stream;
  return FVM_OK;
}
}  // namespace fvm

extern "C" {

int fvm_set_state(fvm_grid* g, const double* src, int src_on_device) {
  if (!g || !src || !g->bound) return FVM_EINVAL;
  const size_t bytes = sizeof(double) * g->elems();
  hipError_t e = hipMemcpyAsync(g->cur, src, bytes,
                                src_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                                g->stream);
  if (e == hipSuccess && !src_on_device) e = hipStreamSynchronize(g->stream);
  g->speeds_valid = false;
  g->me_valid = false;
  return dev_err(e);
}

int fvm_get_state(fvm_grid* g, double* dst, int dst_on_device) {
  if (!g || !dst || !g->bound) return FVM_EINVAL;
  const size_t bytes = sizeof(double) * g->elems();
  hipError_t e = hipMemcpyAsync(dst, g->cur, bytes,
                                dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                                g->stream);
  if (e == hipSuccess && !dst_on_device) e = hipStreamSynchronize(g->stream);
  return dev_err(e);
}

// Points the scratch's dt log at `log` (cap entries, cursor rewound) for the
// steps enqueued next; log == null turns logging off. Every path that
// enqueues steps calls it first, so no step logs into a buffer of an earlier
// run.
static int arm_log(fvm_grid* g, double* log, int cap) {
  if (!log && !g->log_armed) return FVM_OK;
  const int rc = dev_err(launch_set_log(g->scr, 1, log, cap, 1, g->stream));
  if (rc == FVM_OK) g->log_armed = log;
  return rc;
}

// One step launch outside a graph: the step kernel, and for the entropy
// closure the source pass that completes it.
static int enqueue_step(fvm_grid* g, const StepArgs& a) {
  const int km = kernel_model(g->p);
  int rc = dev_err(launch_step(a, km, g->stream));
  if (rc || km != kSprayMaxEnt) return rc;
  MaxEntWarm wm{g->me_lam, g->me_lam && g->me_valid ? 1 : 0, 0};
  rc = dev_err(launch_maxent_source(a, wm, g->stream));
  if (rc == FVM_OK && g->me_lam) g->me_valid = true;
  return rc;
}

static int enqueue_cfl(fvm_grid* g, double* dt_dev) {
  CflArgs a{};
  a.w = g->cur;
  a.scr = g->scr;
  a.dt_out = dt_dev;
  a.g = g->g;
  a.m = g->m;
  const long long cells = static_cast<long long>(g->g.nx) * g->g.ny;
  a.nblocks = static_cast<int>(std::min<long long>(2048, (cells + 255) / 256));
  const int rc = dev_err(launch_cfl(a, g->p.model, g->stream));
  if (rc == FVM_OK) g->speeds_valid = true;
  return rc;
}

int fvm_cfl_dt(fvm_grid* g, double* dt_dev) {
  if (!g || !g->bound) return FVM_EINVAL;
  return enqueue_cfl(g, dt_dev);
}

static int read_scratch(fvm_grid* g, GridScratch* host) {
  hipError_t e = hipStreamSynchronize(g->stream);
  if (e == hipSuccess) e = hipMemcpy(host, g->scr, sizeof(GridScratch), hipMemcpyDeviceToHost);
  return dev_err(e);
}

int fvm_cfl_dt_host(fvm_grid* g, double* dt, double* sx, double* sy) {
  if (!g || !g->bound || !dt) return FVM_EINVAL;
  int rc = enqueue_cfl(g, nullptr);
  if (rc) return rc;
  GridScratch h;
  rc = read_scratch(g, &h);
  if (rc) return rc;
  *dt = h.dt;
  if (sx) *sx = h.cur_sx;
  if (sy) *sy = h.cur_sy;
  return status_from_bits(h.status);
}

int fvm_sync(fvm_grid* g) {
  if (!g || !g->bound) return FVM_EINVAL;
  GridScratch h;
  const int rc = read_scratch(g, &h);
  if (rc) return rc;
  return status_from_bits(h.status);
}

int fvm_get_status(fvm_grid* g, int clear) {
  if (!g || !g->bound) return FVM_EINVAL;
  GridScratch h;
  int rc = read_scratch(g, &h);
  if (rc) return rc;
  rc = status_from_bits(h.status);
  if (clear && h.status) {
    const unsigned int zero = 0;
    const hipError_t e = hipMemcpy(&g->scr->status, &zero, sizeof(zero), hipMemcpyHostToDevice);
    if (e != hipSuccess) return FVM_EDEVICE;
  }
  return rc;
}

int fvm_step(fvm_grid* g, double dt) {
  if (!g || !g->bound) return FVM_EINVAL;
  if (!(dt > 0.0) || !std::isfinite(dt)) return FVM_EINVAL;
  int rc = FVM_OK;
  if (!g->speeds_valid) rc = enqueue_cfl(g, nullptr);
  if (rc == FVM_OK) rc = arm_log(g, nullptr, 0);
  if (rc) return rc;
  StepArgs a = g->step_args(g->cur, g->other(g->cur), kDtFixedCheck);
  a.dt_arg = dt;
  rc = enqueue_step(g, a);
  if (rc == FVM_OK) g->cur = a.wout;
  return rc;
}

static GraphKey graph_key(const fvm_grid* g, int kind, int n, const double* start,
                          const double* dts, int k0, double dt) {
  const bool me_warm = g->me_lam && g->me_valid;
  return GraphKey{kind,   n,      start,  g->other(start), dts, k0,
                  g->rows, g->wpb, g->cpl, dt, g->me_lam, me_warm};
}

// The cached graph of `key`, moved to the front of the cache, or null.
static CachedGraph* find_graph(fvm_grid* g, const GraphKey& key) {
  for (auto it = g->graphs.begin(); it != g->graphs.end(); ++it) {
    if (it->key == key) {
      g->graphs.splice(g->graphs.begin(), g->graphs, it);
      return &g->graphs.front();
    }
  }
  return nullptr;
}

// Builds the graph of `key`: n consecutive steps starting from buffer
// key.start, with step k reading its dt according to the kind.
static int build_graph(fvm_grid* g, const GraphKey& key, hipGraphExec_t* exec) {
  const int kind = key.kind, n = key.nsteps, k0 = key.k0;
  const double* start = key.start;
  const double* dts = key.dts;
  const double dt = key.dt;
  const bool me_warm = key.me_warm;
  CachedGraph c;
  c.key = key;
  if (hipGraphCreate(&c.graph, 0) != hipSuccess) return FVM_EDEVICE;
  hipGraphNode_t prev = nullptr;
  const double* in = start;
  const int km = kernel_model(g->p);
  void* fn = step_kernel_ptr(km, g->p.bc, g->wpb, g->cpl, g->halo.s || g->halo.n);
  std::vector<StepArgs> args(n);
  for (int s = 0; s < n; ++s) {
    double* out = g->other(in);
    args[s] = g->step_args(in, out,
                           kind == 0 ? kDtAdaptive : (kind == 3 ? kDtFixedCheck : kDtArray));
    args[s].dts = dts;
    args[s].dt_arg = dt;
    args[s].k = kind == 2 ? 0 : k0 + s;  // kind 2: dry run, dts = the scratch's zero
    void* kp[] = {&args[s]};
    hipKernelNodeParams np{};
    np.func = fn;
    np.gridDim = dim3(args[s].t.ntiles);
    np.blockDim = dim3(g->wpb * kWave);
    np.sharedMemBytes = 0;
    np.kernelParams = kp;
    np.extra = nullptr;
    hipGraphNode_t node;
    if (hipGraphAddKernelNode(&node, c.graph, prev ? &prev : nullptr, prev ? 1 : 0, &np) !=
        hipSuccess) {
      (void)hipGraphDestroy(c.graph);
      return FVM_EDEVICE;
    }
    prev = node;
    if (km == kSprayMaxEnt) {  // the source pass completes the step
      MaxEntLaunch ml = maxent_launch(args[s]);
      MaxEntWarm wm{g->me_lam, g->me_lam && (me_warm || s > 0) ? 1 : 0, 0};
      void* mp[] = {&args[s], &ml.rule, &wm};
      hipKernelNodeParams sp{};
      sp.func = ml.fn;
      sp.gridDim = ml.grid;
      sp.blockDim = ml.block;
      sp.kernelParams = mp;
      if (hipGraphAddKernelNode(&node, c.graph, &prev, 1, &sp) != hipSuccess) {
        (void)hipGraphDestroy(c.graph);
        return FVM_EDEVICE;
      }
      prev = node;
    }
    in = out;
  }
  if (hipGraphInstantiate(&c.exec, c.graph, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(c.graph);
    return FVM_EDEVICE;
  }
  g->graphs.push_front(c);
  while (g->graphs.size() > kGraphCacheMax) {
    auto& b = g->graphs.back();
    (void)hipGraphExecDestroy(b.exec);
    (void)hipGraphDestroy(b.graph);
    g->graphs.pop_back();
  }
  *exec = c.exec;
  return FVM_OK;
}

// Finds or builds the graph of `n` consecutive steps starting from buffer
// `start`, with step k reading its dt according to `kind`.
static int graph_for(fvm_grid* g, int kind, int n, double* start, const double* dts, int k0,
                     hipGraphExec_t* exec, double dt = 0.0) {
  const GraphKey key = graph_key(g, kind, n, start, dts, k0, dt);
  if (CachedGraph* c = find_graph(g, key)) {
    *exec = c->exec;
    return FVM_OK;
  }
  return build_graph(g, key, exec);
}

// Adaptive and fixed-dt runs: on a miss, builds the graph of every chunk size
// from both ping-pong buffers, so that any later run of this kind and
// configuration only replays.
static int chunk_graph(fvm_grid* g, int kind, int n, double dt, hipGraphExec_t* exec) {
  const GraphKey key = graph_key(g, kind, n, g->cur, nullptr, 0, dt);
  if (CachedGraph* c = find_graph(g, key)) {
    *exec = c->exec;
    return FVM_OK;
  }
  for (double* start : {g->other(g->cur), g->cur}) {
    for (int m : kChunkSizes) {
      if (start == g->cur && m == n) continue;  // built last: it heads the cache
      const GraphKey k = graph_key(g, kind, m, start, nullptr, 0, dt);
      hipGraphExec_t e;
      if (!find_graph(g, k) && build_graph(g, k, &e) != FVM_OK) return FVM_EDEVICE;
    }
  }
  return build_graph(g, key, exec);
}

// The largest chunk size not above `left`.
static int chunk_size(int left) {
  for (int m : kChunkSizes)
    if (m <= left) return m;
  return 1;
}

// A run of adaptive steps on this grid can stay in one workgroup's LDS:
// advection, Euler or the lognormal spray, no halo rows, two states within
// kResidentDoubles.
static bool resident_ok(const fvm_grid* g) {
  if (!g->resident || g->halo.s || g->halo.n) return false;
  if (g->p.model == FVM_SPRAY && g->p.closure != FVM_CLOSURE_LOGNORMAL) return false;
  const long long need = 2LL * fvm_nvar(g->p.model) * g->p.nx * g->p.ny;
  return need <= kResidentDoubles;
}

static int run_steps(fvm_grid* g, int kind, int nsteps, const double* dts, double* log,
                     double dt = 0.0) {
  int rc = FVM_OK;
  // adaptive steps and checked fixed steps read the current state's maxima
  if ((kind == 0 || kind == 3) && !g->speeds_valid) rc = enqueue_cfl(g, nullptr);
  if (rc == FVM_OK) rc = arm_log(g, log, nsteps);
  if (rc) return rc;
  if (kind == 0 && nsteps > 0 && resident_ok(g)) {
    double* other = g->other(g->cur);
    double* last = nsteps % 2 ? other : g->cur;
    double* prev = nsteps % 2 ? g->cur : other;
    const StepArgs a = g->step_args(g->cur, other, kDtAdaptive);
    rc = dev_err(launch_resident_run(a, kernel_model(g->p), last, prev, nsteps, g->stream));
    if (rc) return rc;
    g->cur = last;
    g->speeds_valid = true;
    return FVM_OK;
  }
  int done = 0;
  while (done < nsteps) {
    hipGraphExec_t exec;
    int n;
    if (kind == 0 || kind == 3) {
      n = chunk_size(nsteps - done);
      rc = chunk_graph(g, kind, n, dt, &exec);
    } else {
      n = std::min(kGraphChunk, nsteps - done);
      rc = graph_for(g, kind, n, g->cur, dts, kind == 1 ? done : 0, &exec, dt);
    }
    if (rc) return rc;
    rc = dev_err(hipGraphLaunch(exec, g->stream));
    if (rc) return rc;
    if (n % 2) g->cur = g->other(g->cur);
    if (g->me_lam) g->me_valid = true;
    done += n;
  }
  g->speeds_valid = true;
  return FVM_OK;
}

int fvm_run(fvm_grid* g, int nsteps, double* dts_dev) {
  if (!g || !g->bound || nsteps < 0) return FVM_EINVAL;
  return run_steps(g, 0, nsteps, nullptr, dts_dev);
}

int fvm_run_fixed(fvm_grid* g, int nsteps, double dt) {
  if (!g || !g->bound || nsteps < 0) return FVM_EINVAL;
  if (!(dt > 0.0) || !std::isfinite(dt)) return FVM_EINVAL;
  return run_steps(g, 3, nsteps, nullptr, nullptr, dt);
}

int fvm_run_dts(fvm_grid* g, int nsteps, const double* dts_dev) {
  if (!g || !g->bound || nsteps < 0 || (nsteps > 0 && !dts_dev)) return FVM_EINVAL;
  return run_steps(g, 1, nsteps, dts_dev, nullptr);
}

int fvm_run_ckpt(fvm_grid* g, int nsteps, int ckpt_every, double* const* ckpts,
                 double* dts_dev) {
  if (!g || !g->bound || nsteps < 0 || ckpt_every < 1 || !ckpts) return FVM_EINVAL;
  const int nck = (nsteps + ckpt_every - 1) / ckpt_every;
  for (int s = 0; s < nck; ++s)
    if (!ckpts[s] || ckpts[s] == g->w_a || ckpts[s] == g->w_b) return FVM_EINVAL;
  int rc = FVM_OK;
  if (!g->speeds_valid) rc = enqueue_cfl(g, nullptr);
  if (rc == FVM_OK) rc = arm_log(g, dts_dev, nsteps);
  if (rc) return rc;
  const size_t bytes = sizeof(double) * g->elems();
  if (nck > 0) {
    rc = dev_err(hipMemcpyAsync(ckpts[0], g->cur, bytes, hipMemcpyDeviceToDevice, g->stream));
    if (rc) return rc;
  }
  const double* in = g->cur;
  for (int k = 0; k < nsteps; ++k) {
    double* out;
    if ((k + 1) % ckpt_every == 0 && (k + 1) / ckpt_every < nck)
      out = ckpts[(k + 1) / ckpt_every];
    else
      out = (in == g->w_a) ? g->w_b : g->w_a;
    StepArgs a = g->step_args(in, out, kDtAdaptive);
    rc = enqueue_step(g, a);
    if (rc) return rc;
    in = out;
  }
  if (nsteps > 0 && in != g->w_a && in != g->w_b) {
    // the run ended on a checkpoint buffer: continue from a ping-pong buffer
    rc = dev_err(hipMemcpyAsync(g->w_a, in, bytes, hipMemcpyDeviceToDevice, g->stream));
    if (rc) return rc;
    in = g->w_a;
  }
  g->cur = const_cast<double*>(in);
  return FVM_OK;
}

int fvm_set_tiling(fvm_grid* g, int rows, int wpb) {
  if (!g) return FVM_EINVAL;
  const int r = rows ? rows : g->rows;
  const int w = wpb ? wpb : g->wpb;
  if (!valid_tiling(r, w)) return FVM_EINVAL;
  if (r != g->rows || w != g->wpb) g->clear_graphs();
  g->rows = r;
  g->wpb = w;
  return FVM_OK;
}

// ---- autotuning --------------------------------------------------------------------

}  // extern "C"

namespace {

std::string device_arch() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return "unknown";
  std::string a = prop.gcnArchName;
  const size_t colon = a.find(':');
  return colon == std::string::npos ? a : a.substr(0, colon);
}

bool cache_lookup(const char* path, const std::string& key, int* rows, int* wpb, int* cpl) {
  if (!path) return false;
  std::ifstream in(path);
  std::string line;
  bool found = false;
  while (std::getline(in, line)) {
    const size_t bar = line.find(" | ");
    if (bar == std::string::npos || line.substr(0, bar) != key) continue;
    int r = 0, w = 0, c = 0;
    if (std::sscanf(line.c_str() + bar + 3, "rows=%d wpb=%d cpl=%d", &r, &w, &c) == 3) {
      *rows = r;
      *wpb = w;
      *cpl = c;
      found = true;  // the last entry for a key wins
    }
  }
  return found;
}

void cache_store(const char* path, const std::string& key, int rows, int wpb, int cpl,
                 double us) {
  if (!path) return;
  std::ofstream out(path, std::ios::app);
  out << key << " | rows=" << rows << " wpb=" << wpb << " cpl=" << cpl << " us=" << us << "\n";
}

}  // namespace

// Times `reps` launches of an n-step dry-run graph (dt = 0) in the current
// tiling; returns microseconds per step, or a negative value on error.
static double time_dry(fvm_grid* g, int n, int reps) {
  hipGraphExec_t exec;
  if (arm_log(g, nullptr, 0) != FVM_OK) return -1.0;
  if (graph_for(g, 2, n, g->cur, &g->scr->zero, 0, &exec) != FVM_OK) return -1.0;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return -1.0;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return -1.0;
  }
  double us = -1.0;
  bool ok = hipGraphLaunch(exec, g->stream) == hipSuccess;  // warm-up
  ok = ok && hipEventRecord(e0, g->stream) == hipSuccess;
  for (int r = 0; r < reps && ok; ++r) ok = hipGraphLaunch(exec, g->stream) == hipSuccess;
  ok = ok && hipEventRecord(e1, g->stream) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
  float ms = 0.0f;
  if (ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess) us = 1e3 * ms / (n * reps);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return us;
}

// Times `reps` dry adjoint launches in the current adjoint tiling on
// (w, lam_in -> lam_out); with dt = 0 every cell writes the value it read,
// so the launches move the real traffic and change nothing (with
// lam_in == lam_out they rewrite it in place).
static double time_adjoint_dry(fvm_grid* g, int reps, const double* w, const double* lam_in,
                               double* lam_out) {
  AdjointArgs a{};
  a.w = w;
  a.lam_in = lam_in;
  a.lam_out = lam_out;
  a.dts = nullptr;
  a.dt_arg = 0.0;
  a.g = g->g;
  a.t = adjoint_tiling(g->g, g->adj_rows, g->adj_wpb,
                       adjoint_cpl(g, a.w, a.lam_in, a.lam_out));
  a.m = g->m;
  std::memcpy(a.ghost, g->ghost, sizeof a.ghost);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return -1.0;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return -1.0;
  }
  double us = -1.0;
  bool ok = launch_adjoint(a, g->p.model, g->ug, g->stream) == hipSuccess;  // warm-up
  ok = ok && hipEventRecord(e0, g->stream) == hipSuccess;
  for (int r = 0; r < reps && ok; ++r)
    ok = launch_adjoint(a, g->p.model, g->ug, g->stream) == hipSuccess;
  ok = ok && hipEventRecord(e1, g->stream) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
  float ms = 0.0f;
  if (ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess) us = 1e3 * ms / reps;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return us;
}

// Tuner candidates: a tile shape and lane layout, and its time per launch.
struct TuneCand {
  double us;
  int rows, wpb, cpl;
};

// Two-stage choice among timed candidates: every candidate is timed once
// over a short window, then the kRetime fastest are timed kRounds more times
// over a longer one and the lowest median wins. A short window that follows
// an idle gap can fall into the device's clock ramp, which alone reorders
// candidates a few percent apart. `time(c, reps)` applies candidate c and
// returns its microseconds per launch (< 0 on a device error).
template <class TimeFn>
static int pick_candidate(std::vector<TuneCand>& cands, TimeFn&& time, int reps_long,
                          TuneCand* best) {
  constexpr int kRetime = 6, kRounds = 3;
  if (cands.empty()) return FVM_EINVAL;
  std::stable_sort(cands.begin(), cands.end(),
                   [](const TuneCand& a, const TuneCand& b) { return a.us < b.us; });
  const int n = std::min<int>(kRetime, static_cast<int>(cands.size()));
  *best = cands[0];
  double best_med = 1e300;
  for (int k = 0; k < n; ++k) {
    double t[kRounds];
    for (int r = 0; r < kRounds; ++r) {
      t[r] = time(cands[k], reps_long);
      if (t[r] < 0) return FVM_EDEVICE;
    }
    std::sort(t, t + kRounds);
    if (t[kRounds / 2] < best_med) {
      best_med = t[kRounds / 2];
      *best = cands[k];
      best->us = best_med;
    }
  }
  return FVM_OK;
}

// The adjoint kernel's tile shape and lane layout (advection and Euler),
// timed on (state, lam_in -> lam_out); fvm_autotune passes the
// current state and the other ping-pong buffer, read and written in place.
static int tune_adjoint(fvm_grid* g, const char* cache_path, const std::string& key,
                        const double* state, const double* lam_in, double* lam_out) {
  if (g->p.model == FVM_SPRAY) return FVM_OK;
  int rows = 0, wpb = 0, cpl = 0;
  if (cache_lookup(cache_path, key, &rows, &wpb, &cpl) && valid_tiling(rows, wpb) &&
      (cpl == 1 || cpl == 2)) {
    g->adj_rows = rows;
    g->adj_wpb = wpb;
    g->adj_cpl = cpl;
    return FVM_OK;
  }
  const int wpbs[4] = {1, 2, 4, 8};
  const int rowss[9] = {4, 8, 16, 32, 48, 64, 96, 128, 256};
  auto time = [&](const TuneCand& c, int reps) {
    g->adj_rows = c.rows;
    g->adj_wpb = c.wpb;
    g->adj_cpl = c.cpl;
    return time_adjoint_dry(g, reps, state, lam_in, lam_out);
  };
  std::vector<TuneCand> cands;
  for (int c : {2, 1}) {
    for (int w : wpbs)
      for (int r : rowss) {
        if (r > g->p.ny && r != rowss[0]) continue;
        if (c == 2 && w == 8 && g->p.model == FVM_EULER) continue;  // spills at 2 waves/SIMD
        g->adj_cpl = c;
        // the timed buffers must allow the layout
        if (adjoint_cpl(g, state, lam_in, lam_out) != c) continue;
        TuneCand t{0.0, r, w, c};
        t.us = time(t, 4);
        if (t.us < 0) return FVM_EDEVICE;
        cands.push_back(t);
      }
  }
  TuneCand best{};
  const int rc = pick_candidate(cands, time, 24, &best);
  if (rc) return rc;
  g->adj_rows = best.rows;
  g->adj_wpb = best.wpb;
  g->adj_cpl = best.cpl;
  cache_store(cache_path, key, best.rows, best.wpb, best.cpl, best.us);
  return FVM_OK;
}

extern "C" {

int fvm_autotune_adjoint(fvm_grid* g, const double* w, const double* lam_in, double* lam_out,
                         const char* cache_path) {
  if (!g || !g->bound || !w || !lam_in || !lam_out || lam_in == lam_out) return FVM_EINVAL;
  if (g->p.model == FVM_SPRAY) return FVM_EUNSUPPORTED;
  char kbuf[256];
  std::snprintf(kbuf, sizeof kbuf,
                "%s grid model=%d bc=%d nx=%d ny=%d ld=%d layout=%d adjoint buffers",
                device_arch().c_str(), g->p.model, g->p.bc, g->p.nx, g->p.ny, g->p.ld,
                g->p.layout);
  return tune_adjoint(g, cache_path, kbuf, w, lam_in, lam_out);
}

int fvm_autotune(fvm_grid* g, const char* cache_path) {
  if (!g || !g->bound) return FVM_EINVAL;
  char kbuf[256];
  std::snprintf(kbuf, sizeof kbuf, "%s grid model=%d bc=%d nx=%d ny=%d ld=%d layout=%d%s",
                device_arch().c_str(), g->p.model, g->p.bc, g->p.nx, g->p.ny, g->p.ld,
                g->p.layout, g->p.closure == FVM_CLOSURE_MAXENT ? " maxent" : "");
  const std::string key = kbuf;
  int rows = 0, wpb = 0, cpl = 0;
  if (cache_lookup(cache_path, key, &rows, &wpb, &cpl) && valid_tiling(rows, wpb) &&
      (cpl == 1 || cpl == 2)) {
    g->rows = rows;
    g->wpb = wpb;
    g->cpl_req = cpl;
    g->clear_graphs();
    choose_layout(g);
    return tune_adjoint(g, cache_path, key + " adjoint", g->cur, g->other(g->cur),
                        g->other(g->cur));
  }
  const int cpls[2] = {2, 1};
  const int wpbs[4] = {1, 2, 4, 8};
  const int rowss[10] = {4, 8, 16, 32, 48, 64, 96, 128, 192, 256};
  const int save_req = g->cpl_req;
  auto apply = [&](const TuneCand& c) {
    g->cpl_req = c.cpl;
    choose_layout(g);
    g->rows = c.rows;
    g->wpb = c.wpb;
  };
  // reps: 8-step graphs
  auto time = [&](const TuneCand& c, int reps) {
    apply(c);
    const double us = time_dry(g, 8, reps);
    g->clear_graphs();  // one graph per candidate, not all of them at once
    return us;
  };
  std::vector<TuneCand> cands;
  for (int c : cpls) {
    g->cpl_req = c;
    choose_layout(g);
    if (g->cpl != c) continue;  // the buffers do not allow this layout
    for (int w : wpbs)
      for (int r : rowss) {
        if (r > g->p.ny && r != rowss[0]) continue;
        TuneCand t{0.0, r, w, c};
        t.us = time(t, 2);
        if (t.us < 0) {
          g->clear_graphs();
          return FVM_EDEVICE;
        }
        cands.push_back(t);
      }
  }
  TuneCand best{0.0, g->rows, g->wpb, g->cpl};
  const int prc = cands.empty() ? FVM_OK : pick_candidate(cands, time, 6, &best);
  g->clear_graphs();
  if (prc) return prc;
  const int br = best.rows, bw = best.wpb, bc = best.cpl;
  g->rows = br;
  g->wpb = bw;
  g->cpl_req = save_req ? save_req : bc;
  choose_layout(g);
  g->speeds_valid = true;  // the dry runs recomputed the maxima of the unchanged state
  cache_store(cache_path, key, br, bw, bc, best.us);
  return tune_adjoint(g, cache_path, key + " adjoint", g->cur, g->other(g->cur),
                      g->other(g->cur));
}

int fvm_set_cells_per_lane(fvm_grid* g, int cpl) {
  if (!g || cpl < 0 || cpl > 2) return FVM_EINVAL;
  g->cpl_req = cpl;
  choose_layout(g);
  return FVM_OK;
}

int fvm_get_cells_per_lane(const fvm_grid* g) { return g ? g->cpl : 0; }

int fvm_set_resident_runs(fvm_grid* g, int enable) {
  if (!g) return FVM_EINVAL;
  g->resident = enable != 0;
  return FVM_OK;
}

int fvm_set_adjoint_tiling(fvm_grid* g, int rows, int wpb, int cells_per_lane) {
  if (!g) return FVM_EINVAL;
  const int r = rows ? rows : g->adj_rows;
  const int w = wpb ? wpb : g->adj_wpb;
  const int c = cells_per_lane ? cells_per_lane : g->adj_cpl;
  if (!valid_tiling(r, w) || (c != 1 && c != 2)) return FVM_EINVAL;
  g->adj_rows = r;
  g->adj_wpb = w;
  g->adj_cpl = c;
  return FVM_OK;
}

int fvm_get_tiling(const fvm_grid* g, int* rows, int* wpb) {
  if (!g || !rows || !wpb) return FVM_EINVAL;
  *rows = g->rows;
  *wpb = g->wpb;
  return FVM_OK;
}

// The entropy closure's adjoint step runs in the grid's free ping-pong
// buffer (W* and then mu); none of the step's buffers may be that buffer,
// and with two cells per lane the transport step needs 16-byte alignment.
static bool maxent_adjoint_buffers_ok(const fvm_grid* g, const double* w, const double* lin,
                                      const double* lout) {
  if (kernel_model(g->p) != kSprayMaxEnt) return true;
  const double* ws = g->other(g->cur);
  auto al = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
  if (w == ws || lin == ws || lout == ws) return false;
  return g->cpl != 2 || al(w);
}

// One adjoint step (w, lin -> lout) with dt = dts[k], or dt_arg if dts is
// null. The entropy closure's step is three launches: the transport step
// W -> W* into the free ping-pong buffer ws, the source's adjoint
// mu = lam + dt J_S(W*)^T lam in place there, then the transport's adjoint
// (w, mu -> lout).
static int enqueue_adjoint(fvm_grid* g, const double* w, const double* lin, double* lout,
                           const double* dts, int k, double dt_arg) {
  AdjointArgs a{};
  a.w = w;
  a.lam_in = lin;
  a.lam_out = lout;
  a.dts = dts;
  a.k = k;
  a.dt_arg = dt_arg;
  a.g = g->g;
  a.t = adjoint_tiling(g->g, g->adj_rows, g->adj_wpb, adjoint_cpl(g, a.w, a.lam_in, a.lam_out));
  a.m = g->m;
  std::memcpy(a.ghost, g->ghost, sizeof a.ghost);
  if (kernel_model(g->p) != kSprayMaxEnt)
    return dev_err(launch_adjoint(a, g->p.model, g->ug, g->stream));
  double* ws = g->other(g->cur);
  StepArgs s = g->step_args(w, ws, dts ? kDtArray : kDtValue);
  s.dts = dts;
  s.k = k;
  s.dt_arg = dt_arg;
  int rc = dev_err(launch_step(s, kSprayMaxEnt, g->stream));
  if (rc) return rc;
  AdjointArgs b = a;
  b.w = ws;
  b.lam_out = ws;
  rc = dev_err(launch_maxent_adjoint_source(b, g->ug, g->stream));
  if (rc) return rc;
  AdjointArgs c = a;
  c.lam_in = ws;
  return dev_err(launch_spray_adjoint(c, g->ug, g->stream, false));
}

int fvm_adjoint_step(fvm_grid* g, const double* w, double dt, const double* lam_in,
                     double* lam_out) {
  if (!g || !g->bound || !w || !lam_in || !lam_out || lam_in == lam_out || w == lam_out)
    return FVM_EINVAL;
  if (!adjoint_supported(g)) return FVM_EUNSUPPORTED;
  if (!(dt >= 0.0) || !std::isfinite(dt)) return FVM_EINVAL;
  if (!maxent_adjoint_buffers_ok(g, w, lam_in, lam_out)) return FVM_EINVAL;
  return enqueue_adjoint(g, w, lam_in, lam_out, nullptr, 0, dt);
}

int fvm_adjoint_run(fvm_grid* g, double* const* ckpts, int ckpt_every, const double* dts_dev,
                    int nsteps, double* lam, double* lam_tmp, double* seg_buf) {
  if (!g || !g->bound || !ckpts || ckpt_every < 1 || !dts_dev || nsteps < 0 || !lam ||
      !lam_tmp || lam == lam_tmp)
    return FVM_EINVAL;
  if (ckpt_every > 1 && !seg_buf) return FVM_EINVAL;
  if (!adjoint_supported(g)) return FVM_EUNSUPPORTED;
  const int nck = (nsteps + ckpt_every - 1) / ckpt_every;
  for (int s = 0; s < nck; ++s)
    if (!ckpts[s]) return FVM_EINVAL;
  const size_t state = g->elems();
  if (kernel_model(g->p) == kSprayMaxEnt) {
    // the entropy closure's steps work in the free ping-pong buffer
    const double* ws = g->other(g->cur);
    if (!maxent_adjoint_buffers_ok(g, lam, lam, lam_tmp)) return FVM_EINVAL;
    for (int s = 0; s < nck; ++s)
      if (!maxent_adjoint_buffers_ok(g, ckpts[s], lam, lam_tmp)) return FVM_EINVAL;
    if (seg_buf && ckpt_every > 1) {
      if (!maxent_adjoint_buffers_ok(g, seg_buf, lam, lam_tmp)) return FVM_EINVAL;
      if (ws >= seg_buf && ws < seg_buf + static_cast<size_t>(ckpt_every - 1) * state)
        return FVM_EINVAL;
    }
  }
  if (const int rc = arm_log(g, nullptr, 0)) return rc;  // the recomputed steps log nothing
  double* lin = lam;
  double* lout = lam_tmp;
  for (int s = nck - 1; s >= 0; --s) {
    const int k0 = s * ckpt_every;
    const int k1 = std::min(nsteps, k0 + ckpt_every);
    // recompute W^{k0+1} .. W^{k1-1} into seg_buf[0 .. k1-k0-2]
    const double* in = ckpts[s];
    for (int k = k0; k + 1 < k1; ++k) {
      double* out = seg_buf + static_cast<size_t>(k - k0) * state;
      StepArgs a = g->step_args(in, out, kDtArray);
      a.dts = dts_dev;
      a.k = k;
      int rc = enqueue_step(g, a);
      if (rc) return rc;
      in = out;
    }
    for (int k = k1 - 1; k >= k0; --k) {
      const double* wk = (k == k0) ? ckpts[s] : seg_buf + static_cast<size_t>(k - k0 - 1) * state;
      int rc = enqueue_adjoint(g, wk, lin, lout, dts_dev, k, 0.0);
      if (rc) return rc;
      std::swap(lin, lout);
    }
  }
  // the recompute left the scratch maxima (and the entropy closure's kept
  // multipliers) describing a recomputed state
  g->speeds_valid = false;
  g->me_valid = false;
  if (lin != lam) {
    return dev_err(hipMemcpyAsync(lam, lin, sizeof(double) * state, hipMemcpyDeviceToDevice,
                                  g->stream));
  }
  return FVM_OK;
}

}  // extern "C"

// ---- adaptive run without any allocation -------------------------------------
// fvm_run_noalloc keeps the grid's scratch block (speed maxima, arrival
// counter, next dt, status word, dt-log cursor) in this file-scope device
// array instead of a caller buffer. Host code never passes the array's name
// to a kernel (on the host it is only a stand-in for the symbol): the first
// call on a device looks up the array's device address with
// hipGetSymbolAddress, with that device current, and every launch takes that
// address. Each device holds its own copy until the process ends; calls
// that overlap on one device share it and race.
namespace {

constexpr size_t kNoAllocScratchBytes = sizeof(GridScratch);  // one grid's block
constexpr int kNoAllocMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kNoAllocMaxDevices] = {};

// Device address of `scratch` on device `dev` (current), or null on error.
void* noalloc_scratch(int dev) {
  if (dev < 0 || dev >= kNoAllocMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
    if (reinterpret_cast<uintptr_t>(ptr) & 255) return nullptr;
    g_noalloc_ptr[dev] = ptr;
  }
  return g_noalloc_ptr[dev];
}

// Writes the status code of the sticky bits (FVM_OK, FVM_ENONFINITE,
// FVM_EINVAL) to *out.
__global__ void noalloc_status_kernel(const GridScratch* s, int* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const unsigned int st = s->status;
    *out = (st & kStatusNonFinite) ? FVM_ENONFINITE
                                   : ((st & kStatusCfl) ? FVM_ECFL
                                                        : ((st & kStatusDt) ? FVM_EINVAL : FVM_OK));
  }
}

}  // namespace

extern "C" {

int fvm_run_noalloc(const fvm_params* p, double* w_a, double* w_b, const double* ug,
                    int nsteps, double* dts_dev, int* status_dev, void* stream) {
  if (!valid_params(p) || !w_a || !w_b || w_a == w_b || nsteps < 0) return FVM_EINVAL;
  if ((reinterpret_cast<uintptr_t>(w_a) & 7) || (reinterpret_cast<uintptr_t>(w_b) & 7))
    return FVM_EINVAL;
  if ((p->model == FVM_SPRAY) != (ug != nullptr)) return FVM_EINVAL;
  if (p->bc == FVM_DIRICHLET || p->closure != FVM_CLOSURE_LOGNORMAL) return FVM_EUNSUPPORTED;
  if (fvm_scratch_bytes(p) > kNoAllocScratchBytes) return FVM_EINVAL;  // beyond the array
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return FVM_EDEVICE;
  GridScratch* scr = static_cast<GridScratch*>(noalloc_scratch(dev));
  if (!scr) return FVM_EDEVICE;
  hipStream_t st = static_cast<hipStream_t>(stream);

  const GridGeom geom = grid_geometry(*p);
  const ModelConsts mc = model_consts(*p);
  auto al16 = [](const void* q) { return (reinterpret_cast<uintptr_t>(q) & 15) == 0; };
  const int cpl = p->ld % 2 == 0 && al16(w_a) && al16(w_b) && (!ug || al16(ug)) ? 2 : 1;
  int rows = kDefaultRows, wpb = kDefaultWpb;
  default_tiling(*p, cpl, &rows, &wpb);

  // clear the block (a kernel, not a memset), maxima and dt of w_a, arm the log
  int rc = dev_err(launch_clear_scratch(scr, 1, st));
  if (rc) return rc;
  CflArgs c{};
  c.w = w_a;
  c.scr = scr;
  c.g = geom;
  c.m = mc;
  const long long cells = static_cast<long long>(p->nx) * p->ny;
  c.nblocks = static_cast<int>(std::min<long long>(2048, (cells + 255) / 256));
  rc = dev_err(launch_cfl(c, p->model, st));
  if (rc == FVM_OK) rc = dev_err(launch_set_log(scr, 1, dts_dev, nsteps, 1, st));
  if (rc) return rc;
  StepArgs a{};
  a.ug = ug;
  a.scr = scr;
  a.mode = kDtAdaptive;
  a.g = geom;
  a.t = tiling(geom, rows, wpb, cpl);
  a.m = mc;
  const double* in = w_a;
  for (int k = 0; k < nsteps; ++k) {
    double* out = in == w_a ? w_b : w_a;
    a.win = in;
    a.wout = out;
    rc = dev_err(launch_step(a, p->model, st));
    if (rc) return rc;
    in = out;
  }
  if (status_dev) {
    hipLaunchKernelGGL(noalloc_status_kernel, dim3(1), dim3(64), 0, st, scr, status_dev);
    rc = dev_err(hipGetLastError());
  }
  return rc;
}

}  // extern "C"
