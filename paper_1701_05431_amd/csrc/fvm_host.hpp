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

}  // namespace fvm
