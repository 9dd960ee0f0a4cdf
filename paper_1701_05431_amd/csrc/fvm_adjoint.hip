// fvm_adjoint.hip -- the adjoint kernels of advection and Euler (one strip
// per wave, in either lane layout) and the launch of every model's adjoint;
// the device code is in fvm_adjoint.hpp (the spray's in fvm_adjoint_spray.hpp).
#include <hip/hip_runtime.h>

#include "../../include/fvm.h"
#include "fvm_adjoint.hpp"
#include "fvm_internal.hpp"
#include "fvm_models.hpp"
#include "fvm_step.hpp"

namespace fvm {

template <class M, int BC, int WPB, int CPL>
__global__ __launch_bounds__(WPB * kWave) void adjoint_kernel(AdjointArgs a) {
  const M m(a.m);
  const double dt = a.dts ? a.dts[a.k] : a.dt_arg;
  const double mux = dt / a.g.dx, muy = dt / a.g.dy;
  // each XCD walks a contiguous range of tiles, as in the forward step, so
  // vertically adjacent tiles share its L2 for their halo rows
  const int tile = xcd_tile(blockIdx.x, a.t.ntiles);
  const int tx = tile % a.t.tiles_x, ty = tile / a.t.tiles_x;
  const int wave = wave_index();
  const int j0 = ty * a.t.rows;
  const int j1 = min(j0 + a.t.rows, a.g.ny);
  if constexpr (CPL == 2) {
    const int xs = (tx * WPB + wave) * 2 * kWave;
    if (xs >= a.g.nx) return;  // the whole wave
    if (xs + 2 * kWave <= a.g.nx)
      adjoint_strip2<M, BC, false>(m, a, xs, j0, j1, mux, muy);
    else
      adjoint_strip2<M, BC, true>(m, a, xs, j0, j1, mux, muy);
  } else {
    const int xs = (tx * WPB + wave) * kOutPerWave;
    if (xs >= a.g.nx) return;
    // tiles of odd rows march down (vertical neighbours meet at their
    // shared rows)
    if (ty & 1)
      adjoint_strip1<M, BC, true>(m, a, xs, j0, j1, mux, muy);
    else
      adjoint_strip1<M, BC, false>(m, a, xs, j0, j1, mux, muy);
  }
}

template <class M, int BC, int CPL>
static void* adj_fn_wpb(int wpb) {
  switch (wpb) {
    case 1: return reinterpret_cast<void*>(&adjoint_kernel<M, BC, 1, CPL>);
    case 2: return reinterpret_cast<void*>(&adjoint_kernel<M, BC, 2, CPL>);
    case 4: return reinterpret_cast<void*>(&adjoint_kernel<M, BC, 4, CPL>);
    case 8: return reinterpret_cast<void*>(&adjoint_kernel<M, BC, 8, CPL>);
    default: return nullptr;
  }
}

template <class M, int CPL>
static void* adj_fn_bc(int bc, int wpb) {
  switch (bc) {
    case kPeriodic: return adj_fn_wpb<M, kPeriodic, CPL>(wpb);
    case kTransmissive: return adj_fn_wpb<M, kTransmissive, CPL>(wpb);
    case kDirichlet: return adj_fn_wpb<M, kDirichlet, CPL>(wpb);
    default: return nullptr;
  }
}

void* adjoint_kernel_ptr(int model, int bc, int wpb, int cpl) {
  if (model == 0) return cpl == 2 ? adj_fn_bc<AdjAdv, 2>(bc, wpb) : adj_fn_bc<AdjAdv, 1>(bc, wpb);
  if (model == 1)
    return cpl == 2 ? adj_fn_bc<AdjEuler, 2>(bc, wpb) : adj_fn_bc<AdjEuler, 1>(bc, wpb);
  return nullptr;
}

hipError_t launch_spray_adjoint(const AdjointArgs& a, const double* ug, hipStream_t st,
                                bool src);

hipError_t launch_adjoint(const AdjointArgs& a, int model, const double* ug, hipStream_t st) {
  if (model == FVM_SPRAY) return launch_spray_adjoint(a, ug, st, true);
  void* f = adjoint_kernel_ptr(model, a.g.bc, a.t.wpb, a.t.cpl);
  if (!f) return hipErrorInvalidValue;
  AdjointArgs copy = a;
  void* args[] = {&copy};
  return hipLaunchKernel(f, dim3(a.t.ntiles), dim3(a.t.wpb * kWave), args, 0, st);
}

}  // namespace fvm
