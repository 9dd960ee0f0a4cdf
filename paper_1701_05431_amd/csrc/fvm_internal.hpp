// fvm_internal.hpp -- launch-argument structures shared by the host library
// and the kernels. Plain data only (passed to kernels by value).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

struct fvm_params;

namespace fvm {

constexpr int kWave = 64;       // CDNA wavefront width
constexpr int kOutPerWave = 62; // cells an adjoint strip updates (lanes 0 and 63: halo)
constexpr int kMaxVar = 6;      // largest nVar (spray)

// Kernel families: the three models (fvm_params.model) and the spray with
// the entropy-maximising closure (a transport step, then a source pass).
enum : int { kSprayMaxEnt = 3 };

// Boundary conditions (template argument BC of the kernels).
enum : int { kPeriodic = 0, kTransmissive = 1, kDirichlet = 2 };
// Sides of the domain, in the order of the Dirichlet ghost states.
enum : int { kWest = 0, kEast = 1, kSouth = 2, kNorth = 3 };

// Sticky device status bits.
enum : unsigned int {
  kStatusNonFinite = 1u,  // NaN/inf speed or a non-physical cell
  kStatusCfl = 2u,        // fixed-dt step failed the CFL check
  kStatusDt = 4u,         // adaptive dt not positive (all speeds zero, no dt_max)
};

// Time-step source of a step launch.
enum : int {
  kDtAdaptive = 0,  // dt from the device scratch (previous finalize)
  kDtFixedCheck = 1,// dt from the argument, checked against eq. CFL_cond
  kDtArray = 2,     // dt = dts[k]
  kDtValue = 3,     // dt from the argument, unchecked (adjoint recomputation)
};

// Per-grid device scratch (256-byte aligned, cleared by the init kernel).
// The dt log of a run lives here too, set by a small kernel before the run's
// steps, so that cached graphs of steps do not depend on the log buffer.
struct alignas(256) GridScratch {
  unsigned long long smax[2];  // running maxima (bit patterns) of the state being produced
  unsigned int arrive;         // arrival counter of the current launch
  unsigned int status;         // sticky status bits
  unsigned int nstep;          // dt-log cursor
  unsigned int pad0;
  double dt;                   // dt of the next adaptive step
  double cur_sx, cur_sy;       // finalized maxima of the current state
  double zero;                 // always 0: the dt of the tuner's dry-run steps
  double pad1;
  double* log;                 // dt log of the current run (null: none)
  int log_cap;                 // entries the log holds
  int log_stride;              // elements between consecutive logged dts
};
static_assert(sizeof(GridScratch) == 256, "scratch layout");

// Model constants.
struct ModelConsts {
  double gamma, gm1;          // Euler
  double ax, ay;              // advection
  double K, inv_theta;        // spray (inv_theta = 0 for no drag)
  double s_eps, log_s_eps;    // spray closure
};

// Geometry and policy of one grid. Variable v of cell (i, j) sits at
// v * plane + j * ld + i: the planar layout has ld = row pitch and
// plane = pitch * ny, the row-interleaved layout ld = nVar * pitch and
// plane = pitch. The spray gas velocity (2 variables) uses uld / uplane.
struct GridGeom {
  int nx, ny, ld, bc;
  size_t plane;
  double dx, dy;              // lx/nx, ly/ny
  double cfl, dt_max;
  double hmin;                // min(dx, dy) for the fixed-dt check
  size_t uplane;
  int uld;
  int rld;                    // pitch of one variable's row (the caller's ld)
};

// Rows j = -1 (s) and j = ny (n) read from the caller's buffers instead of
// the boundary rule, one row each with variable v of column i at
// [v * rld + i]: the halo rows a slab of a larger grid receives from its
// neighbours. A null pointer leaves that side to the boundary condition.
struct Halo {
  const double* s;
  const double* n;
};

// Geometry of a validated parameter set (fvm_api.hip).
GridGeom grid_geometry(const fvm_params& p);

// Cells a wave strip updates: 64 with one cell per lane, 128 with two.
__host__ __device__ constexpr int strip_width(int cpl) { return cpl == 2 ? 2 * kWave : kWave; }

// LDS doubles of the resident run (two states of nVar x nx x ny): 144 KiB
constexpr int kResidentDoubles = 18432;

// Tile decomposition of one grid for a launch.
struct Tiling {
  int rows;        // rows marched per strip
  int wpb;         // wave strips per workgroup
  int cpl;         // cells per lane (1 or 2)
  int tiles_x;     // ceil(nx / (strip_width * wpb))
  int tiles_y;     // ceil(ny / rows)
  int ntiles;
};

struct StepArgs {
  const double* win;
  double* wout;
  const double* ug;           // spray gas velocity (2 planes) or null
  GridScratch* scr;
  int mode;
  int k;                      // kDtArray index
  double dt_arg;              // kDtFixedCheck
  const double* dts;          // kDtArray
  GridGeom g;
  Tiling t;
  ModelConsts m;
  double ghost[4 * kMaxVar];  // Dirichlet states: ghost[side * kMaxVar + v]
  Halo halo;
};

struct CflArgs {
  const double* w;
  GridScratch* scr;
  double* dt_out;             // nullable device pointer
  GridGeom g;
  ModelConsts m;
  int nblocks;
};

struct AdjointArgs {
  const double* w;            // forward state W^n
  const double* lam_in;       // lambda^{n+1}
  double* lam_out;            // lambda^n
  const double* dts;          // dt = dts[k] if dts != null, else dt_arg
  int k;
  int pad;
  double dt_arg;
  GridGeom g;
  Tiling t;
  ModelConsts m;
  double ghost[4 * kMaxVar];  // Dirichlet states: ghost[side * kMaxVar + v]
};

// ---- batches ---------------------------------------------------------------

struct BatchGrid {            // per-grid record in device memory
  size_t offset;              // element offset of the grid inside the packed buffers
  GridGeom g;
  int strips_x;               // wave strips across the grid
  int tiles_y;                // row blocks
  int rows;                   // rows per block (the last block may be shorter)
  int nstrips;                // strips_x * tiles_y wave strips, numbered row-major
  int nitems;                 // work items: groups of WPB consecutive strips
  int item0;                  // first work item of the grid
  int user;                   // the caller's index of the grid
  int cpl;                    // cells per lane of the grid's strips
};

struct BatchScratch {         // header of the batch scratch
  unsigned int queue;         // next work item
  unsigned int arrive;        // blocks done with the launch
  unsigned int status;
  unsigned int nstep;
  unsigned int pad[60];
};
static_assert(sizeof(BatchScratch) == 256, "batch scratch layout");

struct BatchArgs {
  const double* win;
  double* wout;
  const BatchGrid* grids;     // device array of n records
  GridScratch* gscr;          // device array of n per-grid scratch blocks
  BatchScratch* bscr;
  int ngrids;                 // records sorted by item0 (tallest row blocks first)
  int nitems;                 // work items of all grids
  double dt_scale;            // 1; 0 for the tuner's dry runs (state unchanged)
  ModelConsts m;
};

// The entropy-maximising spray source pass (fvm_maxent.hip) takes its
// quadrature rule as a kernel argument.
struct MaxEntRule {  // 8-point Gauss-Legendre rule on [0, 1]
  double x[8], w[8];
};

}  // namespace fvm
