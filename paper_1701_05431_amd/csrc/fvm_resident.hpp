// fvm_resident.hpp -- device code of a whole adaptive run of a small grid in
// one workgroup (the state lives in LDS between steps).
//
// A grid whose two states fit in one workgroup's LDS (the 64 x 64 advection
// case, Euler grids up to about 48 x 48) is bound by launch latency when
// every step is its own launch. Here one workgroup holds the state and the
// next state in LDS and runs all the steps of the run: per step every thread
// updates its cells (Sec. 2.2.1 eq. VF_scheme, and for the spray the source
// of Sec. 2.2.2), the workgroup reduces the new state's speeds, and thread 0
// computes the next dt (eq. CFL_cond), logs the one just used and flags a
// non-finite state or a non-positive dt, exactly as the last workgroup of a
// step launch does. Each face flux is evaluated with the same arguments,
// each update with the same operations, and the maxima and dt by the same
// code as in the marching strips, so a resident run is bitwise the run of
// step launches. At the end the last two states go back to the two
// ping-pong buffers and the dt, maxima, status and log cursor to the grid's
// scratch block.
#pragma once

#include <hip/hip_runtime.h>

#include <cfloat>

#include "fvm_internal.hpp"
#include "fvm_models.hpp"
#include "fvm_step.hpp"

namespace fvm {
namespace res {

// Threads of a resident run: 1024 for advection; 512 for Euler and the spray,
// whose per-cell registers (the cells' neighbour indices kept for the whole
// run, the flux and source arithmetic) need more than the 128 per lane that
// 16 waves leave
template <class M>
constexpr int threads() {
  return M::NV == 1 ? 1024 : 512;
}

// Where a cell's state and its four neighbours' live: LDS indices into a
// compact state s[v * ncell + j * nx + i] (neighbours through the boundary
// rule: periodic wrap, transmissive copy), or -1 - side for a Dirichlet
// ghost. Set up once per run, used every step.
struct Cell {
  int at, west, east, south, north;
  size_t uc;  // the cell in the gas-velocity planes
};

template <int BC>
__device__ __forceinline__ int neighbour_at(const GridGeom& g, int j, int i) {
  if constexpr (BC == kDirichlet) {
    if (i < 0) return -1 - kWest;
    if (i >= g.nx) return -1 - kEast;
    if (j < 0) return -1 - kSouth;
    if (j >= g.ny) return -1 - kNorth;
  }
  return row_index<BC>(j, g.ny) * g.nx + col_index<BC>(i, g.nx);
}

template <int BC>
__device__ __forceinline__ Cell cell_at(const GridGeom& g, int c) {
  const int j = c / g.nx, i = c % g.nx;
  Cell r;
  r.at = c;
  r.west = neighbour_at<BC>(g, j, i - 1);
  r.east = neighbour_at<BC>(g, j, i + 1);
  r.south = neighbour_at<BC>(g, j - 1, i);
  r.north = neighbour_at<BC>(g, j + 1, i);
  r.uc = ucell(g, j, i);
  return r;
}

template <int NV>
__device__ __forceinline__ void load_at(const double* s, int ncell, const double* gh, int at,
                                        double* w) {
  if (at < 0) {
#pragma unroll
    for (int v = 0; v < NV; ++v) w[v] = gh[(-1 - at) * kMaxVar + v];
    return;
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) w[v] = s[v * ncell + at];
}

// The update of cell r from state `s` into `o` (ugx, ugy: its gas velocity,
// spray only), folding the new state's speeds into (bx, by).
template <class M>
__device__ __forceinline__ void update_cell(const M& m, const double* gh, const double* s,
                                            double* o, int ncell, const Cell& r, double ugx,
                                            double ugy, double mux, double muy, double dt,
                                            unsigned long long& bx, unsigned long long& by) {
  constexpr int NV = M::NV;
  using Prim = typename M::Prim;
  double W[NV], N[NV], Fw[NV], Fe[NV], Gs[NV], Gn[NV];
  Prim P, Q;
  load_at<NV>(s, ncell, gh, r.at, W);
  m.prim(W, P);
  load_at<NV>(s, ncell, gh, r.west, N);
  m.prim(N, Q);
  m.template flux<0>(N, Q, W, P, Fw);
  load_at<NV>(s, ncell, gh, r.east, N);
  m.prim(N, Q);
  m.template flux<0>(W, P, N, Q, Fe);
  load_at<NV>(s, ncell, gh, r.south, N);
  m.prim(N, Q);
  m.template flux<1>(N, Q, W, P, Gs);
  load_at<NV>(s, ncell, gh, r.north, N);
  m.prim(N, Q);
  m.template flux<1>(W, P, N, Q, Gn);
  double Wo[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) Wo[v] = W[v] - fma(mux, Fe[v] - Fw[v], muy * (Gn[v] - Gs[v]));
  if constexpr (M::kSource) m.source(Wo, ugx, ugy, dt);
#pragma unroll
  for (int v = 0; v < NV; ++v) o[v * ncell + r.at] = Wo[v];
  double sx, sy;
  m.speeds(Wo, sx, sy);
  bx = umax64(bx, bits(sx));
  by = umax64(by, bits(sy));
}

// Cells per thread of a resident run of model M (two states in the LDS).
template <class M>
constexpr int max_cells() {
  return (kResidentDoubles / (2 * M::NV) + threads<M>() - 1) / threads<M>();
}

// The run's bookkeeping after a step with maxima (sx, sy) and dt `used`:
// the status bits and the next dt, as finalize_grid computes them.
__device__ __forceinline__ double next_step_dt(const GridGeom& g, double sx, double sy,
                                               unsigned int& st) {
  if (!(sx <= DBL_MAX) || !(sy <= DBL_MAX)) st |= kStatusNonFinite;
  const double dtn = next_dt(g, sx, sy);
  if (!(dtn > 0.0)) st |= kStatusDt;
  return dtn;
}

}  // namespace res
}  // namespace fvm
