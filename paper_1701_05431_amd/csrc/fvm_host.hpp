// fvm_host.hpp -- host-side declarations shared between the library's
// translation units (not seen by the kernels' device code).
#pragma once

#include "../../include/fvm.h"
#include "fvm_internal.hpp"

namespace fvm {

// What the output stage needs to know of a bound grid (fvm_api.hip).
struct GridView {
  fvm_params p;
  GridGeom g;
  int nv;
  const double* cur;   // buffer holding the current state
  hipStream_t stream;  // the stream the grid's work is enqueued on
};
int grid_view(const fvm_grid* g, GridView* v);

// The entropy-maximising spray source pass (fvm_maxent.hip): launched after
// the transport-only step kernel, on the step's output buffer.
struct MaxEntLaunch {
  void* fn;
  dim3 grid, block;
  MaxEntRule rule;
};
// Multipliers of the previous source pass, per cell (dense planes
// lam[(k * ny + j) * nx + i], k = 0..3): Newton starts from them when `warm`
// is set and writes the converged ones back; lam may be null.
struct MaxEntWarm {
  double* lam;
  int warm;
  int pad;
};
MaxEntLaunch maxent_launch(const StepArgs& a);
hipError_t launch_maxent_source(const StepArgs& a, const MaxEntWarm& wm, hipStream_t st);

}  // namespace fvm
