// fvm_kernels.hip -- gfx950 kernels of the fused first-order finite-volume step.
//
// One launch performs one whole time step (Sec. 2.2.1 eq. VF_scheme + the
// split source of Sec. 2.2.2 + the time-step reduction of eq. CFL_cond) on
// a grid held as FP64 rows in HBM (one row of nx values per variable and
// grid row, planar or row-interleaved).
//
// Work decomposition. A wave (64 lanes) owns a strip of 128 consecutive
// columns (two cells per lane, 16-byte accesses) or 64 (one per lane) and
// marches up a range of rows. Each lane keeps its cells of the current row
// and of the rows in flight in registers; the rows below and above come from
// the march (each y-face flux is computed once and carried to the next row),
// the left/right neighbours from the adjacent lanes by DPP moves (each x-face
// flux is computed once and handed to the lane on its right), and the two
// faces at the strip's ends from a halo cell that lanes 0 and 63 load. This
// replaces the paper's overlap strips and its copyOverlaps / internalResiduals
// / borderResiduals / update tasks: a subdomain border is an ordinary
// neighbour read straight from HBM, and every cell goes through the same code
// path, so the result does not depend on how the grid is split into
// subdomains or tiles.
//
// Each state is read once and written once per step (plus the halo rows and
// columns of each strip). The new state's speeds are reduced in the same
// pass (wave shuffle, workgroup LDS, one 64-bit atomicMax per workgroup on
// the bit patterns, which orders non-negative doubles and puts NaN above
// +inf), and the last workgroup to arrive computes the next time step on the
// device.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cstdint>

#include "fvm_internal.hpp"
#include "fvm_models.hpp"
#include "fvm_step.hpp"

namespace fvm {

// One wave strip of the CPL layout (1: 64 cells per wave, any pitch; 2: 128
// cells per wave, 16-byte aligned accesses; down: march the rows from the
// top of the tile, CPL 2 only).
// (gh: the Dirichlet ghost states, BC == kDirichlet only; HALO: rows -1 and
// ny may come from the halo buffers)
template <class M, int BC, int CPL, bool HALO>
__device__ __forceinline__ void strip(const M& m, const double* __restrict__ win,
                                      double* __restrict__ wout, const double* __restrict__ ug,
                                      const GridGeom& g, int xs, int j0, int j1, double mux,
                                      double muy, double dt, unsigned long long& bx,
                                      unsigned long long& by, const double* gh,
                                      const Halo& halo, bool down) {
  if (xs >= g.nx) return;
  if (CPL == 1) {
    if (xs + kWave <= g.nx)
      march_strip1<M, BC, false, HALO>(m, win, wout, ug, g, xs, j0, j1, mux, muy, dt, bx, by,
                                       gh, halo);
    else
      march_strip1<M, BC, true, HALO>(m, win, wout, ug, g, xs, j0, j1, mux, muy, dt, bx, by, gh,
                                      halo);
  } else if (xs + 2 * kWave <= g.nx) {
    if (down)
      march_strip2<M, BC, false, M::kPrefetch2, HALO, true>(m, win, wout, ug, g, xs, j0, j1,
                                                            mux, muy, dt, bx, by, gh, halo);
    else
      march_strip2<M, BC, false, M::kPrefetch2, HALO>(m, win, wout, ug, g, xs, j0, j1, mux,
                                                      muy, dt, bx, by, gh, halo);
  } else {
    if (down)
      march_strip2<M, BC, true, M::kPrefetch2, HALO, true>(m, win, wout, ug, g, xs, j0, j1,
                                                           mux, muy, dt, bx, by, gh, halo);
    else
      march_strip2<M, BC, true, M::kPrefetch2, HALO>(m, win, wout, ug, g, xs, j0, j1, mux, muy,
                                                     dt, bx, by, gh, halo);
  }
}

template <class M, int BC, int WPB, int CPL, bool HALO>
__global__ FVM_STEP_BOUNDS(WPB) void step_kernel(StepArgs a) {
  const M m(a.m);
  bool cfl_fail;
  const double dt = launch_dt(a, cfl_fail);
  const double dt_eff = cfl_fail ? 0.0 : dt;
  const double mux = dt_eff / a.g.dx, muy = dt_eff / a.g.dy;
  const int tile = xcd_tile(blockIdx.x, a.t.ntiles);
  const int tx = tile % a.t.tiles_x, ty = tile / a.t.tiles_x;
  const int wave = wave_index();
  const int xs = (tx * WPB + wave) * strip_width(CPL);
  const int j0 = ty * a.t.rows;
  const int j1 = min(j0 + a.t.rows, a.g.ny);
  unsigned long long bx = 0, by = 0;
  // two-cells-per-lane strips of odd tile rows march down: vertically
  // adjacent tiles then read the rows they share at about the same time
  strip<M, BC, CPL, HALO>(m, a.win, a.wout, a.ug, a.g, xs, j0, j1, mux, muy, dt_eff, bx, by,
                          a.ghost, a.halo, (ty & 1) != 0);
  if constexpr (M::kCommit) {
    if (block_commit<WPB>(bx, by, a.scr, gridDim.x) && threadIdx.x == 0) {
      if (cfl_fail) atomicOr(&a.scr->status, kStatusCfl);
      finalize_grid(a.scr, a.g, dt_eff, true, nullptr);
    }
  }
}

// Speed maxima of a state and the adaptive dt (the checkTimeStep task).
template <class M>
__global__ __launch_bounds__(256) void cfl_kernel(CflArgs a) {
  const M m(a.m);
  unsigned long long bx = 0, by = 0;
  const long long ncell = static_cast<long long>(a.g.nx) * a.g.ny;
  for (long long c = blockIdx.x * 256ll + threadIdx.x; c < ncell; c += 256ll * gridDim.x) {
    const int j = static_cast<int>(c / a.g.nx), i = static_cast<int>(c % a.g.nx);
    double w[M::NV];
#pragma unroll
    for (int v = 0; v < M::NV; ++v) w[v] = a.w[v * a.g.plane + static_cast<size_t>(j) * a.g.ld + i];
    double sx, sy;
    m.speeds(w, sx, sy);
    bx = umax64(bx, bits(sx));
    by = umax64(by, bits(sy));
  }
  if (block_commit<4>(bx, by, a.scr, gridDim.x) && threadIdx.x == 0)
    finalize_grid(a.scr, a.g, 0.0, false, a.dt_out);
}

__global__ void clear_scratch_kernel(GridScratch* s, int n) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) {
    GridScratch z = {};
    s[k] = z;
  }
}

// Sets the dt log of the next run on n grids' scratch blocks: grid k logs
// into base + k every `stride` elements, at most cap entries; base == null
// turns logging off. Rewinds the cursors.
__global__ void set_log_kernel(GridScratch* s, int n, double* base, int cap, int stride) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) {
    s[k].log = base ? base + k : nullptr;
    s[k].log_cap = base ? cap : 0;
    s[k].log_stride = stride;
    s[k].nstep = 0;
  }
}

}  // namespace fvm

// ---- host-side launch helpers (used by fvm_api.hip) --------------------------------
namespace fvm {

using StepFn = void (*)(StepArgs);

template <class M, int BC, int CPL, bool HALO>
static StepFn step_fn_wpb(int wpb) {
  switch (wpb) {
    case 1: return &step_kernel<M, BC, 1, CPL, HALO>;
    case 2: return &step_kernel<M, BC, 2, CPL, HALO>;
    case 4: return &step_kernel<M, BC, 4, CPL, HALO>;
    case 8: return &step_kernel<M, BC, 8, CPL, HALO>;
    default: return nullptr;
  }
}

// Halo rows are combined with periodic or transmissive x-boundaries only.
template <class M, int CPL>
static StepFn step_fn_cpl(int bc, int wpb, bool halo) {
  switch (bc) {
    case kPeriodic:
      return halo ? step_fn_wpb<M, kPeriodic, CPL, true>(wpb)
                  : step_fn_wpb<M, kPeriodic, CPL, false>(wpb);
    case kTransmissive:
      return halo ? step_fn_wpb<M, kTransmissive, CPL, true>(wpb)
                  : step_fn_wpb<M, kTransmissive, CPL, false>(wpb);
    case kDirichlet: return halo ? nullptr : step_fn_wpb<M, kDirichlet, CPL, false>(wpb);
    default: return nullptr;
  }
}

template <class M>
static StepFn step_fn_bc(int bc, int wpb, int cpl, bool halo) {
  return cpl == 2 ? step_fn_cpl<M, 2>(bc, wpb, halo) : step_fn_cpl<M, 1>(bc, wpb, halo);
}

// The transport-only spray step (entropy-maximising closure): periodic and
// transmissive boundaries, no halo rows.
template <int CPL>
static StepFn transport_fn(int bc, int wpb, bool halo) {
  if (halo) return nullptr;
  if (bc == kPeriodic) return step_fn_wpb<SprayTransport, kPeriodic, CPL, false>(wpb);
  if (bc == kTransmissive) return step_fn_wpb<SprayTransport, kTransmissive, CPL, false>(wpb);
  return nullptr;
}

void* step_kernel_ptr(int model, int bc, int wpb, int cpl, bool halo) {
  StepFn f = nullptr;
  if (model == 0) f = step_fn_bc<Adv>(bc, wpb, cpl, halo);
  else if (model == 1) f = step_fn_bc<Euler>(bc, wpb, cpl, halo);
  else if (model == 2) f = step_fn_bc<Spray>(bc, wpb, cpl, halo);
  else if (model == kSprayMaxEnt)
    f = cpl == 2 ? transport_fn<2>(bc, wpb, halo) : transport_fn<1>(bc, wpb, halo);
  return reinterpret_cast<void*>(f);
}

hipError_t launch_step(const StepArgs& a, int model, hipStream_t st) {
  void* f = step_kernel_ptr(model, a.g.bc, a.t.wpb, a.t.cpl, a.halo.s || a.halo.n);
  if (!f) return hipErrorInvalidValue;
  StepArgs copy = a;
  void* args[] = {&copy};
  return hipLaunchKernel(f, dim3(a.t.ntiles), dim3(a.t.wpb * kWave), args, 0, st);
}

hipError_t launch_cfl(const CflArgs& a, int model, hipStream_t st) {
  CflArgs copy = a;
  void* args[] = {&copy};
  void* f = nullptr;
  if (model == 0) f = reinterpret_cast<void*>(&cfl_kernel<Adv>);
  else if (model == 1) f = reinterpret_cast<void*>(&cfl_kernel<Euler>);
  else if (model == 2) f = reinterpret_cast<void*>(&cfl_kernel<Spray>);
  if (!f) return hipErrorInvalidValue;
  return hipLaunchKernel(f, dim3(a.nblocks), dim3(256), args, 0, st);
}

hipError_t launch_clear_scratch(GridScratch* s, int n, hipStream_t st) {
  hipLaunchKernelGGL(clear_scratch_kernel, dim3((n + 63) / 64), dim3(64), 0, st, s, n);
  return hipGetLastError();
}

hipError_t launch_set_log(GridScratch* s, int n, double* base, int cap, int stride,
                          hipStream_t st) {
  hipLaunchKernelGGL(set_log_kernel, dim3((n + 63) / 64), dim3(64), 0, st, s, n, base, cap,
                     stride);
  return hipGetLastError();
}

}  // namespace fvm
