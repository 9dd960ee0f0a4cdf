// fvm_batch.hip -- many independent grids of uneven sizes advanced together.
//
// One persistent launch per time step walks a work list of (grid, group of
// strips) items, longest items (tallest row blocks) first, handed out by an
// atomic queue, so that short items fill the gaps the long ones leave, the
// step ends on short ones and no launch is smaller than the chip. A grid's
// wave strips (the single-grid kernel's strips, over row blocks of
// near-equal height, at most the tuned `rows`) are numbered row-major and an
// item is WPB consecutive strips of one grid, one per wave: a grid narrower
// than a workgroup stacks its waves over several row blocks instead of
// leaving them idle, and a small grid takes shorter blocks so that it still
// has a strip for every wave. The device code per
// strip is the single-grid kernel's, so a grid's result is bit-for-bit the
// one of a single-grid launch. Each grid keeps its own adaptive dt: the item's
// workgroup folds its speeds into the grid's maxima and the last item of a
// grid computes that grid's next dt. The last workgroup of the launch rewinds
// the queue.
//
// The reference schedule -- one launch of the single-grid kernel per grid per
// time step -- is available as fvm_batch_run_per_grid.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <list>
#include <new>
#include <numeric>
#include <cstdio>
#include <fstream>
#include <string>
#include <vector>

#include "../../include/fvm.h"
#include "fvm_internal.hpp"
#include "fvm_models.hpp"
#include "fvm_step.hpp"

namespace fvm {

void* step_kernel_ptr(int model, int bc, int wpb, int cpl, bool halo);
hipError_t launch_cfl(const CflArgs& a, int model, hipStream_t st);
hipError_t launch_clear_scratch(GridScratch* s, int n, hipStream_t st);
hipError_t launch_set_log(GridScratch* s, int n, double* base, int cap, int stride,
                          hipStream_t st);

__global__ void batch_clear_kernel(BatchScratch* b, GridScratch* g, int n) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k == 0) {
    BatchScratch z = {};
    *b = z;
  }
  if (k < n) {
    GridScratch z = {};
    g[k] = z;
  }
}

// PERSIST: a resident set of workgroups takes items from the queue until it
// runs dry; otherwise (grouped launch) workgroup b does item b and the
// hardware dispatcher balances the load. NARROW: every grid runs one cell
// per lane, and the two-cell strips are left out of the kernel (about 150
// registers per lane for the Euler strips instead of about 245, so three
// waves per SIMD instead of two, and the last strip of a grid idles at most
// 63 lanes instead of 127).
template <class M, int BC, int WPB, bool PERSIST, bool NARROW>
__global__ FVM_STEP_BOUNDS(WPB) void batch_kernel(BatchArgs a) {
  // both lane layouts live in the mixed kernel, so the Euler strips keep one
  // row of loads in flight (not two) to stay within 256 registers per lane
  // (two rows in flight, even with the one-cell strips left out, spill)
  constexpr int kPF = M::NV >= 4 ? 1 : M::kPrefetch2;
  const M m(a.m);
  const int wave = wave_index();
  __shared__ int s_item;
  for (;;) {
    int item;
    if constexpr (PERSIST) {
      // the workgroup's next item, through LDS: every thread reads it
      // after the barrier
      if (threadIdx.x == 0) s_item = static_cast<int>(atomicAdd(&a.bscr->queue, 1u));
      __syncthreads();
      item = s_item;
      __syncthreads();
    } else {
      item = static_cast<int>(blockIdx.x);
    }
    if (item >= a.nitems) break;
    int lo = 0, hi = a.ngrids - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (a.grids[mid].item0 <= item) lo = mid; else hi = mid - 1;
    }
    const BatchGrid G = a.grids[lo];
    GridScratch* s = a.gscr + G.user;
    const double dt = s->dt * a.dt_scale;
    const double mux = dt / G.g.dx, muy = dt / G.g.dy;
    const int k = (item - G.item0) * WPB + wave;  // this wave's strip
    unsigned long long bx = 0, by = 0;
    if (k < G.nstrips) {
      const int sx = k % G.strips_x, ty = k / G.strips_x;
      const bool wide_grid = !NARROW && G.cpl == 2;  // uniform across the workgroup
      const int xs = sx * (wide_grid ? strip_width(2) : strip_width(1));
      // a two-cells-per-lane grid's last strip with at most 64 columns left
      // runs one cell per lane (bitwise the same cells, half the idle lanes)
      const bool wide = wide_grid && xs + kWave < G.g.nx;
      const int j0 = ty * G.rows;
      const int j1 = min(j0 + G.rows, G.g.ny);
      const double* win = a.win + G.offset;
      double* wout = a.wout + G.offset;
      if (!wide && xs + kWave <= G.g.nx)
        march_strip1<M, BC, false>(m, win, wout, nullptr, G.g, xs, j0, j1, mux, muy, dt, bx, by);
      else if (!wide)
        march_strip1<M, BC, true>(m, win, wout, nullptr, G.g, xs, j0, j1, mux, muy, dt, bx, by);
      else if (xs + 2 * kWave <= G.g.nx)
        march_strip2<M, BC, false, kPF>(m, win, wout, nullptr, G.g, xs, j0, j1, mux, muy, dt, bx,
                                        by);
      else
        march_strip2<M, BC, true, kPF>(m, win, wout, nullptr, G.g, xs, j0, j1, mux, muy, dt, bx,
                                       by);
    }
    if (block_commit<WPB>(bx, by, s, static_cast<unsigned int>(G.nitems)) && threadIdx.x == 0)
      finalize_grid(s, G.g, dt, true, nullptr);
    if constexpr (!PERSIST) break;
  }
  if (PERSIST && threadIdx.x == 0) {
    __threadfence();
    const unsigned int t = atomicAdd(&a.bscr->arrive, 1u);
    if (t == gridDim.x - 1) {
      atomicExch(&a.bscr->queue, 0u);
      atomicExch(&a.bscr->arrive, 0u);
    }
  }
}

template <class M, int BC, bool P, bool N>
static void* batch_fn_wpb(int wpb) {
  switch (wpb) {
    case 1: return reinterpret_cast<void*>(&batch_kernel<M, BC, 1, P, N>);
    case 2: return reinterpret_cast<void*>(&batch_kernel<M, BC, 2, P, N>);
    case 4: return reinterpret_cast<void*>(&batch_kernel<M, BC, 4, P, N>);
    case 8: return reinterpret_cast<void*>(&batch_kernel<M, BC, 8, P, N>);
    default: return nullptr;
  }
}

template <class M, bool P, bool N>
static void* batch_fn_bc(int bc, int wpb) {
  return bc == 0 ? batch_fn_wpb<M, 0, P, N>(wpb) : batch_fn_wpb<M, 1, P, N>(wpb);
}

template <class M>
static void* batch_fn(int bc, int wpb, bool persist, bool narrow) {
  if (persist)
    return narrow ? batch_fn_bc<M, true, true>(bc, wpb) : batch_fn_bc<M, true, false>(bc, wpb);
  return narrow ? batch_fn_bc<M, false, true>(bc, wpb) : batch_fn_bc<M, false, false>(bc, wpb);
}

static void* batch_kernel_ptr(int model, int bc, int wpb, bool persist, bool narrow) {
  if (model == 0) return batch_fn<Adv>(bc, wpb, persist, narrow);
  if (model == 1) return batch_fn<Euler>(bc, wpb, persist, narrow);
  return nullptr;
}

}  // namespace fvm

using namespace fvm;

namespace {

int berr(hipError_t e) { return e == hipSuccess ? FVM_OK : FVM_EDEVICE; }

constexpr int kBatchChunks[6] = {32, 16, 8, 4, 2, 1};  // steps per persistent-run graph
constexpr size_t kBatchGraphCacheMax = 16;

struct BatchGraph {
  int kind;  // 0 persistent, 1 per grid
  int nsteps;
  const double* start;
  int rows, wpb, cpl_max;
  bool persist, fit;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

}  // namespace

struct fvm_batch {
  int n = 0;
  int model = 0, bc = 0, nv = 0;
  std::vector<fvm_params> p;
  std::vector<size_t> offsets;
  std::vector<int> order;        // grids by decreasing area
  ModelConsts m{};
  int rows = 32, wpb = 2;
  bool persist = true;           // persistent workgroups or one per item
  bool fit = false;              // row blocks chosen to fill whole workgroups
  int cpl_max = 2;               // 2: two cells per lane where the pitch is even; 1: one
  bool narrow = false;           // every grid runs one cell per lane
  double* w_a = nullptr;
  double* w_b = nullptr;
  double* cur = nullptr;
  unsigned char* scratch = nullptr;
  const double* log_armed = nullptr;  // dt log the per-grid scratch currently points to
  hipStream_t stream = nullptr;
  bool bound = false, speeds_valid = false;
  int nitems = 0;
  int nblocks = 0;               // persistent workgroups
  std::vector<BatchGrid> recs;   // in processing order (per-grid scratch: by caller index)
  std::list<BatchGraph> graphs;

  ~fvm_batch() { clear_graphs(); }
  void clear_graphs() {
    for (auto& c : graphs) {
      if (c.exec) (void)hipGraphExecDestroy(c.exec);
      if (c.graph) (void)hipGraphDestroy(c.graph);
    }
    graphs.clear();
  }
  BatchScratch* bscr() const { return reinterpret_cast<BatchScratch*>(scratch); }
  GridScratch* gscr() const {
    return reinterpret_cast<GridScratch*>(scratch + sizeof(BatchScratch));
  }
  BatchGrid* drecs() const {
    return reinterpret_cast<BatchGrid*>(scratch + sizeof(BatchScratch) +
                                        sizeof(GridScratch) * static_cast<size_t>(n));
  }
  double* other(const double* w) const { return w == w_a ? w_b : w_a; }

  static constexpr int kMinRows = 8;
  static constexpr int kStripCostRows = 4;  // a strip's start-up, in rows

  // (re)builds the work list for the current tiling
  void plan() {
    recs.clear();
    for (int k : order) {
      BatchGrid r{};
      r.offset = offsets[k];
      r.user = k;
      const GridGeom g = grid_geometry(p[k]);
      r.g = g;
      // two cells per lane needs 16-byte aligned rows: an even pitch (the
      // grid offsets are multiples of 32 elements, the buffers 256-byte
      // aligned)
      r.cpl = cpl_max == 2 && p[k].ld % 2 == 0 ? 2 : 1;
      const int w = strip_width(r.cpl);
      r.strips_x = (g.nx + w - 1) / w;
      // row blocks of near-equal height (a workgroup waits for its longest
      // strip), at most `rows` high. A grid with fewer strips than a
      // workgroup has waves is cut into shorter blocks, down to kMinRows, so
      // that its item keeps the waves busy. With `fit`, the block count is
      // the one that occupies the fewest wave-rows, counting the idle waves
      // of a grid's last, partly filled item and a fixed cost per strip, so
      // a grid whose strip count does not divide into whole workgroups takes
      // somewhat shorter blocks instead
      const int ty0 = (g.ny + rows - 1) / rows;
      const int tyfill = std::max(ty0, std::min((wpb + r.strips_x - 1) / r.strips_x,
                                                g.ny / kMinRows));
      const int tymax = fit ? std::max(ty0, std::min(std::max(4 * ty0, tyfill), g.ny / kMinRows))
                            : ty0;
      int ty = fit ? ty0 : tyfill;
      long long best = -1;
      for (int t = ty0; fit && t <= tymax; ++t) {
        const long long ns = static_cast<long long>(r.strips_x) * t;
        const long long cost =
            (ns + wpb - 1) / wpb * wpb * ((g.ny + t - 1) / t + kStripCostRows);
        if (best < 0 || cost < best) {
          best = cost;
          ty = t;
        }
      }
      r.rows = (g.ny + ty - 1) / ty;
      r.tiles_y = (g.ny + r.rows - 1) / r.rows;
      r.nstrips = r.strips_x * r.tiles_y;
      r.nitems = (r.nstrips + wpb - 1) / wpb;
      recs.push_back(r);
    }
    // the queue hands out the longest items (tallest blocks) first, so the
    // step ends on short ones; equal heights keep the larger grid first
    std::stable_sort(recs.begin(), recs.end(),
                     [](const BatchGrid& x, const BatchGrid& y) { return x.rows > y.rows; });
    int item = 0;
    narrow = true;
    for (auto& r : recs) {
      r.item0 = item;
      item += r.nitems;
      narrow = narrow && r.cpl == 1;
    }
    nitems = item;
  }
};

extern "C" {

int fvm_batch_create(int n, const fvm_params* p, const size_t* offsets, fvm_batch** out) {
  if (!out) return FVM_EINVAL;
  *out = nullptr;
  if (n < 1 || !p || !offsets) return FVM_EINVAL;
  for (int k = 0; k < n; ++k) {
    if (fvm_validate(&p[k]) != FVM_OK) return FVM_EINVAL;
    if (p[k].model == FVM_SPRAY || p[k].bc == FVM_DIRICHLET) return FVM_EUNSUPPORTED;
    if (p[k].model != p[0].model || p[k].bc != p[0].bc) return FVM_EINVAL;
    if (p[k].gamma != p[0].gamma || p[k].ax != p[0].ax || p[k].ay != p[0].ay) return FVM_EINVAL;
    if (offsets[k] % 32 != 0) return FVM_EINVAL;
  }
  const int nv = fvm_nvar(p[0].model);
  // the grids must not overlap
  std::vector<int> by_off(n);
  std::iota(by_off.begin(), by_off.end(), 0);
  std::sort(by_off.begin(), by_off.end(), [&](int a, int b) { return offsets[a] < offsets[b]; });
  for (int q = 0; q + 1 < n; ++q) {
    const int a = by_off[q], b = by_off[q + 1];
    const size_t end = offsets[a] + static_cast<size_t>(nv) * p[a].ld * p[a].ny;
    if (end > offsets[b]) return FVM_EINVAL;
  }
  fvm_batch* b = new (std::nothrow) fvm_batch();
  if (!b) return FVM_EINVAL;
  b->n = n;
  b->model = p[0].model;
  b->bc = p[0].bc;
  b->nv = nv;
  b->p.assign(p, p + n);
  b->offsets.assign(offsets, offsets + n);
  b->order.resize(n);
  std::iota(b->order.begin(), b->order.end(), 0);
  std::stable_sort(b->order.begin(), b->order.end(), [&](int x, int y) {
    return static_cast<long long>(p[x].nx) * p[x].ny > static_cast<long long>(p[y].nx) * p[y].ny;
  });
  fvm_params q = p[0];
  ModelConsts m{};
  m.gamma = q.gamma;
  m.gm1 = q.gamma - 1.0;
  m.ax = q.ax;
  m.ay = q.ay;
  b->m = m;
  b->plan();
  *out = b;
  return FVM_OK;
}

int fvm_batch_destroy(fvm_batch* b) {
  delete b;
  return FVM_OK;
}

size_t fvm_batch_scratch_bytes(const fvm_batch* b) {
  if (!b) return 0;
  size_t s = sizeof(BatchScratch) + sizeof(GridScratch) * static_cast<size_t>(b->n) +
             sizeof(BatchGrid) * static_cast<size_t>(b->n);
  return (s + 255) / 256 * 256;
}

static int upload_records(fvm_batch* b) {
  hipError_t e = hipMemcpyAsync(b->drecs(), b->recs.data(), sizeof(BatchGrid) * b->recs.size(),
                                hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  return berr(e);
}

// The persistent launch's workgroup count: as many as fit on the device at
// once for the kernel of the current tiling and layout.
static int size_resident_set(fvm_batch* b) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return FVM_EDEVICE;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return FVM_EDEVICE;
  void* f = batch_kernel_ptr(b->model, b->bc, b->wpb, true, b->narrow);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, b->wpb * kWave, 0) != hipSuccess)
    return FVM_EDEVICE;
  b->nblocks = std::max(1, cus * std::max(1, per_cu));
  return FVM_OK;
}

int fvm_batch_bind(fvm_batch* b, double* w_a, double* w_b, void* scratch, void* stream) {
  if (!b || !w_a || !w_b || !scratch || w_a == w_b) return FVM_EINVAL;
  if (reinterpret_cast<uintptr_t>(scratch) & 255) return FVM_EINVAL;
  if ((reinterpret_cast<uintptr_t>(w_a) & 255) || (reinterpret_cast<uintptr_t>(w_b) & 255))
    return FVM_EINVAL;
  b->clear_graphs();
  b->w_a = w_a;
  b->w_b = w_b;
  b->cur = w_a;
  b->scratch = static_cast<unsigned char*>(scratch);
  b->stream = static_cast<hipStream_t>(stream);
  b->bound = true;
  b->speeds_valid = false;
  b->log_armed = nullptr;
  if (size_resident_set(b) != FVM_OK) return FVM_EDEVICE;
  hipLaunchKernelGGL(batch_clear_kernel, dim3((b->n + 63) / 64), dim3(64), 0, b->stream,
                     b->bscr(), b->gscr(), b->n);
  if (hipGetLastError() != hipSuccess) return FVM_EDEVICE;
  return upload_records(b);
}

int fvm_batch_set_tiling(fvm_batch* b, int rows, int wpb) {
  if (!b) return FVM_EINVAL;
  const int r = rows ? rows : b->rows;
  const int w = wpb ? wpb : b->wpb;
  if (r < 1 || r > 4096 || !(w == 1 || w == 2 || w == 4 || w == 8)) return FVM_EINVAL;
  b->clear_graphs();
  b->rows = r;
  b->wpb = w;
  b->plan();
  if (!b->bound) return FVM_OK;
  if (size_resident_set(b) != FVM_OK) return FVM_EDEVICE;
  return upload_records(b);
}

int fvm_batch_cfl(fvm_batch* b) {
  if (!b || !b->bound) return FVM_EINVAL;
  for (int q = 0; q < b->n; ++q) {
    const BatchGrid& r = b->recs[q];
    CflArgs a{};
    a.w = b->cur + r.offset;
    a.scr = b->gscr() + r.user;
    a.g = r.g;
    a.m = b->m;
    const long long cells = static_cast<long long>(r.g.nx) * r.g.ny;
    a.nblocks = static_cast<int>(std::min<long long>(1024, (cells + 255) / 256));
    if (launch_cfl(a, b->model, b->stream) != hipSuccess) return FVM_EDEVICE;
  }
  b->speeds_valid = true;
  return FVM_OK;
}

// Points every grid's dt log at log + k (stride n, cap entries, cursors
// rewound) for the steps enqueued next; null turns logging off.
static int arm_batch_log(fvm_batch* b, double* log, int cap) {
  if (!log && !b->log_armed) return FVM_OK;
  if (launch_set_log(b->gscr(), b->n, log, cap, b->n, b->stream) != hipSuccess)
    return FVM_EDEVICE;
  b->log_armed = log;
  return FVM_OK;
}

// The cached graph of `nsteps` steps of `kind` from buffer `start` in the
// current tiling and schedule, moved to the front of the cache, or null.
static BatchGraph* find_batch_graph(fvm_batch* b, int kind, int nsteps, const double* start) {
  for (auto it = b->graphs.begin(); it != b->graphs.end(); ++it) {
    if (it->kind == kind && it->nsteps == nsteps && it->start == start &&
        it->rows == b->rows && it->wpb == b->wpb && it->persist == b->persist &&
        it->fit == b->fit && it->cpl_max == b->cpl_max) {
      b->graphs.splice(b->graphs.begin(), b->graphs, it);
      return &b->graphs.front();
    }
  }
  return nullptr;
}

static int build_batch_graph(fvm_batch* b, int kind, int nsteps, const double* start,
                             hipGraphExec_t* exec) {
  BatchGraph c;
  c.kind = kind;
  c.nsteps = nsteps;
  c.start = start;
  c.rows = b->rows;
  c.wpb = b->wpb;
  c.persist = b->persist;
  c.fit = b->fit;
  c.cpl_max = b->cpl_max;
  if (hipGraphCreate(&c.graph, 0) != hipSuccess) return FVM_EDEVICE;
  hipGraphNode_t prev = nullptr;
  const double* in = start;
  auto add = [&](void* fn, dim3 grid, dim3 block, void* arg) -> bool {
    void* kp[] = {arg};
    hipKernelNodeParams np{};
    np.func = fn;
    np.gridDim = grid;
    np.blockDim = block;
    np.sharedMemBytes = 0;
    np.kernelParams = kp;
    np.extra = nullptr;
    hipGraphNode_t node;
    if (hipGraphAddKernelNode(&node, c.graph, prev ? &prev : nullptr, prev ? 1 : 0, &np) !=
        hipSuccess)
      return false;
    prev = node;
    return true;
  };
  bool ok = true;
  for (int s = 0; s < nsteps && ok; ++s) {
    double* out = b->other(in);
    if (kind != 1) {  // 0: persistent launch; 2: its dry run (dt scaled to 0)
      BatchArgs a{};
      a.win = in;
      a.wout = out;
      a.grids = b->drecs();
      a.gscr = b->gscr();
      a.bscr = b->bscr();
      a.ngrids = b->n;
      a.nitems = b->nitems;
      a.dt_scale = kind == 2 ? 0.0 : 1.0;
      a.m = b->m;
      ok = add(batch_kernel_ptr(b->model, b->bc, b->wpb, b->persist, b->narrow),
               dim3(b->persist ? std::min(b->nblocks, b->nitems) : b->nitems),
               dim3(b->wpb * kWave), &a);
    } else {
      for (int q = 0; q < b->n && ok; ++q) {
        const BatchGrid& r = b->recs[q];
        StepArgs a{};
        a.win = in + r.offset;
        a.wout = out + r.offset;
        a.scr = b->gscr() + r.user;
        a.mode = kDtAdaptive;
        a.g = r.g;
        // the single-grid kernel's workgroup tiles
        a.t.rows = r.rows;
        a.t.wpb = b->wpb;
        a.t.cpl = r.cpl;
        a.t.tiles_x = (r.strips_x + b->wpb - 1) / b->wpb;
        a.t.tiles_y = r.tiles_y;
        a.t.ntiles = a.t.tiles_x * a.t.tiles_y;
        a.m = b->m;
        ok = add(step_kernel_ptr(b->model, b->bc, b->wpb, r.cpl, false), dim3(a.t.ntiles),
                 dim3(b->wpb * kWave),
                 &a);
      }
    }
    in = out;
  }
  if (!ok || hipGraphInstantiate(&c.exec, c.graph, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(c.graph);
    return FVM_EDEVICE;
  }
  b->graphs.push_front(c);
  while (b->graphs.size() > kBatchGraphCacheMax) {
    auto& x = b->graphs.back();
    (void)hipGraphExecDestroy(x.exec);
    (void)hipGraphDestroy(x.graph);
    b->graphs.pop_back();
  }
  *exec = c.exec;
  return FVM_OK;
}

static int batch_graph(fvm_batch* b, int kind, int nsteps, hipGraphExec_t* exec) {
  if (BatchGraph* c = find_batch_graph(b, kind, nsteps, b->cur)) {
    *exec = c->exec;
    return FVM_OK;
  }
  return build_batch_graph(b, kind, nsteps, b->cur, exec);
}

// Persistent runs are cut into graphs of 32, 16, 8, 4, 2 and 1 steps; a miss
// builds every chunk size from both ping-pong buffers, so a later run of any
// length only replays cached graphs.
static int batch_chunk_graph(fvm_batch* b, int n, hipGraphExec_t* exec) {
  if (BatchGraph* c = find_batch_graph(b, 0, n, b->cur)) {
    *exec = c->exec;
    return FVM_OK;
  }
  for (const double* start : {static_cast<const double*>(b->other(b->cur)),
                              static_cast<const double*>(b->cur)}) {
    for (int m : kBatchChunks) {
      if (start == b->cur && m == n) continue;  // built last: it heads the cache
      hipGraphExec_t e;
      if (!find_batch_graph(b, 0, m, start) && build_batch_graph(b, 0, m, start, &e) != FVM_OK)
        return FVM_EDEVICE;
    }
  }
  return build_batch_graph(b, 0, n, b->cur, exec);
}

static int batch_run(fvm_batch* b, int kind, int nsteps, double* log) {
  if (!b || !b->bound || nsteps < 0) return FVM_EINVAL;
  int rc = FVM_OK;
  if (!b->speeds_valid) rc = fvm_batch_cfl(b);
  if (rc == FVM_OK) rc = arm_batch_log(b, log, nsteps);
  if (rc) return rc;
  int done = 0;
  while (done < nsteps) {
    const int left = nsteps - done;
    int n = std::min(2, left);
    hipGraphExec_t exec;
    if (kind == 0) {
      n = 1;
      for (int m : kBatchChunks)
        if (m <= left) {
          n = m;
          break;
        }
      rc = batch_chunk_graph(b, n, &exec);
    } else {
      rc = batch_graph(b, kind, n, &exec);
    }
    if (rc) return rc;
    if (hipGraphLaunch(exec, b->stream) != hipSuccess) return FVM_EDEVICE;
    if (n % 2) b->cur = b->other(b->cur);
    done += n;
  }
  return FVM_OK;
}

int fvm_batch_run(fvm_batch* b, int nsteps, double* dts_dev) {
  return batch_run(b, 0, nsteps, dts_dev);
}

int fvm_batch_run_per_grid(fvm_batch* b, int nsteps, double* dts_dev) {
  return batch_run(b, 1, nsteps, dts_dev);
}

int fvm_batch_current(const fvm_batch* b, double** w) {
  if (!b || !w || !b->bound) return FVM_EINVAL;
  *w = b->cur;
  return FVM_OK;
}

// Chooses the batch tiling and schedule by timing dry launches (dt scaled to
// 0, states unchanged) of every candidate; see fvm_autotune.
int fvm_batch_autotune(fvm_batch* b, const char* cache_path) {
  if (!b || !b->bound) return FVM_EINVAL;
  unsigned long long h = 1469598103934665603ull;  // FNV-1a over the grid shapes
  for (const auto& p : b->p)
    for (int x : {p.nx, p.ny, p.ld, p.layout}) {
      h ^= static_cast<unsigned long long>(x);
      h *= 1099511628211ull;
    }
  int dev = 0;
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
    arch = prop.gcnArchName;
    arch = arch.substr(0, arch.find(':'));
  }
  char kbuf[256];
  std::snprintf(kbuf, sizeof kbuf, "%s batch model=%d bc=%d n=%d shapes=%016llx", arch.c_str(),
                b->model, b->bc, b->n, h);
  const std::string key = kbuf;
  if (cache_path) {
    std::ifstream in(cache_path);
    std::string line;
    int r = 0, w = 0, ps = 1, ft = 0, cl = 2, found = 0;
    while (std::getline(in, line)) {
      const size_t bar = line.find(" | ");
      if (bar == std::string::npos || line.substr(0, bar) != key) continue;
      int rr = 0, ww = 0, pp = 1, ff = 0, cc = 2;
      const int got = std::sscanf(line.c_str() + bar + 3, "rows=%d wpb=%d persist=%d fit=%d cpl=%d",
                                  &rr, &ww, &pp, &ff, &cc);
      if (got >= 4 && (cc == 1 || cc == 2)) {  // lines without a layout: two cells per lane
        r = rr, w = ww, ps = pp, ft = ff, cl = got == 5 ? cc : 2;
        found = 1;
      }
    }
    if (found) {
      b->persist = ps != 0;
      b->fit = ft != 0;
      b->cpl_max = cl;
      return fvm_batch_set_tiling(b, r, w);
    }
  }
  if (!b->speeds_valid) {
    const int rc = fvm_batch_cfl(b);
    if (rc) return rc;
  }
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return FVM_EDEVICE;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return FVM_EDEVICE;
  }
  double best = 1e300;
  int br = b->rows, bw = b->wpb, bc = b->cpl_max;
  bool bp = b->persist, bf = b->fit;
  int rc = FVM_OK;
  for (int c = 0; c < 32 && !rc; ++c) {
    const int cl = c < 16 ? 2 : 1;  // two cells per lane, then one
    const bool ps = c % 16 < 8;     // persistent, then grouped launches
    const bool ft = c % 2 == 1;
    const int w = 1 << ((c / 2) % 4);
    b->persist = ps;
    b->fit = ft;
    b->cpl_max = cl;
    for (int r : {8, 16, 32, 48, 64, 96, 128, 192, 256}) {
      rc = fvm_batch_set_tiling(b, r, w);
      if (rc == FVM_OK) rc = arm_batch_log(b, nullptr, 0);
      if (rc) break;
      hipGraphExec_t exec;
      const int n = 4;
      rc = batch_graph(b, 2, n, &exec);
      if (rc) break;
      bool ok = hipGraphLaunch(exec, b->stream) == hipSuccess;
      ok = ok && hipEventRecord(e0, b->stream) == hipSuccess;
      for (int k = 0; k < 2 && ok; ++k) ok = hipGraphLaunch(exec, b->stream) == hipSuccess;
      ok = ok && hipEventRecord(e1, b->stream) == hipSuccess &&
           hipEventSynchronize(e1) == hipSuccess;
      float ms = 0.0f;
      if (!ok || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        rc = FVM_EDEVICE;
        break;
      }
      const double us = 1e3 * ms / (2 * n);
      if (us < best) {
        best = us;
        br = r;
        bw = w;
        bp = ps;
        bf = ft;
        bc = cl;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  b->persist = bp;
  b->fit = bf;
  b->cpl_max = bc;
  rc = fvm_batch_set_tiling(b, br, bw);
  if (rc == FVM_OK && cache_path) {
    std::ofstream out(cache_path, std::ios::app);
    out << key << " | rows=" << br << " wpb=" << bw << " persist=" << (bp ? 1 : 0)
        << " fit=" << (bf ? 1 : 0) << " cpl=" << bc << " us=" << best << "\n";
  }
  return rc;
}

int fvm_batch_set_schedule(fvm_batch* b, int persistent, int fit_blocks) {
  if (!b) return FVM_EINVAL;
  b->persist = persistent != 0;
  b->fit = fit_blocks != 0;
  return fvm_batch_set_tiling(b, b->rows, b->wpb);
}

int fvm_batch_set_layout(fvm_batch* b, int cells_per_lane) {
  if (!b || (cells_per_lane != 1 && cells_per_lane != 2)) return FVM_EINVAL;
  b->cpl_max = cells_per_lane;
  return fvm_batch_set_tiling(b, b->rows, b->wpb);
}

int fvm_batch_sync(fvm_batch* b) {
  if (!b || !b->bound) return FVM_EINVAL;
  if (hipStreamSynchronize(b->stream) != hipSuccess) return FVM_EDEVICE;
  std::vector<GridScratch> h(b->n);
  if (hipMemcpy(h.data(), b->gscr(), sizeof(GridScratch) * b->n, hipMemcpyDeviceToHost) !=
      hipSuccess)
    return FVM_EDEVICE;
  unsigned int st = 0;
  for (const auto& x : h) st |= x.status;
  if (st & kStatusNonFinite) return FVM_ENONFINITE;
  if (st & kStatusDt) return FVM_EINVAL;
  return FVM_OK;
}

}  // extern "C"
