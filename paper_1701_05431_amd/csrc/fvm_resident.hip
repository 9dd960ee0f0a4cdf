// fvm_resident.hip -- the resident run kernel (device code and rationale in
// fvm_resident.hpp): one workgroup (1024 threads for advection, 512 for Euler
// and the spray) runs every adaptive step of a run of a grid whose two
// states fit in its LDS.
#include <hip/hip_runtime.h>

#include "fvm_internal.hpp"
#include "fvm_models.hpp"
#include "fvm_resident.hpp"
#include "fvm_step.hpp"

namespace fvm {

namespace {

template <class M, int BC>
__global__ __launch_bounds__(res::threads<M>()) void resident_run_kernel(StepArgs a,
                                                                         double* w_last,
                                                                         double* w_prev,
                                                                         int nsteps) {
  constexpr int NV = M::NV;
  constexpr int kThreads = res::threads<M>(), kWaves = kThreads / kWave;
  __shared__ double lds[kResidentDoubles];
  __shared__ unsigned long long red[2][kWaves];
  __shared__ double s_dt;
  const M m(a.m);
  const GridGeom& g = a.g;
  const int ncell = g.nx * g.ny;
  const int tid = static_cast<int>(threadIdx.x);
  const int wave = wave_index();
  double* A = lds;
  double* B = lds + NV * ncell;
  for (int c = tid; c < ncell; c += kThreads) {
    const size_t at = static_cast<size_t>(c / g.nx) * g.ld + c % g.nx;
#pragma unroll
    for (int v = 0; v < NV; ++v) A[v * ncell + c] = a.win[v * g.plane + at];
  }
  // this thread's cells (tid, tid + 1024, ...) and their neighbours, once
  constexpr int kCells = res::max_cells<M>();
  res::Cell cells[kCells];
  double ugx[kCells], ugy[kCells];
#pragma unroll
  for (int q = 0; q < kCells; ++q) {
    const int c = tid + q * kThreads;
    cells[q] = res::cell_at<BC>(g, c < ncell ? c : 0);
    ugx[q] = ugy[q] = 0.0;
    if constexpr (M::kSource) {
      if (c < ncell) {
        ugx[q] = a.ug[cells[q].uc];
        ugy[q] = a.ug[g.uplane + cells[q].uc];
      }
    }
  }
  GridScratch* const s = a.scr;
  double dt = s->dt;
  double sx = s->cur_sx, sy = s->cur_sy;
  // the dt log, read once (thread 0 keeps it in registers)
  double* const log = s->log;
  const unsigned int cap = static_cast<unsigned int>(s->log_cap);
  const size_t stride = static_cast<size_t>(s->log_stride);
  unsigned int st = 0, n = s->nstep;
  __syncthreads();
  for (int k = 0; k < nsteps; ++k) {
    const double mux = dt / g.dx, muy = dt / g.dy;
    unsigned long long bx = 0, by = 0;
#pragma unroll
    for (int q = 0; q < kCells; ++q)
      if (tid + q * kThreads < ncell)
        res::update_cell<M>(m, a.ghost, A, B, ncell, cells[q], ugx[q], ugy[q], mux, muy, dt, bx,
                            by);
    bx = wave_max64(bx);
    by = wave_max64(by);
    if ((tid & (kWave - 1)) == 0) {
      red[0][wave] = bx;
      red[1][wave] = by;
    }
    __syncthreads();
    if (tid == 0) {
      unsigned long long mx = red[0][0], my = red[1][0];
#pragma unroll
      for (int q = 1; q < kWaves; ++q) {
        mx = umax64(mx, red[0][q]);
        my = umax64(my, red[1][q]);
      }
      sx = __longlong_as_double(static_cast<long long>(mx));
      sy = __longlong_as_double(static_cast<long long>(my));
      const double dtn = res::next_step_dt(g, sx, sy, st);
      if (log) {  // the dt this step used, as the step launches log it
        if (n < cap) log[static_cast<size_t>(n) * stride] = dt;
        ++n;
      }
      s_dt = dtn;
    }
    __syncthreads();
    dt = s_dt;
    double* t = A;
    A = B;
    B = t;
  }
  // state n to the buffer that becomes current, state n - 1 to the other
  for (int c = tid; c < ncell; c += kThreads) {
    const size_t at = static_cast<size_t>(c / g.nx) * g.ld + c % g.nx;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      w_last[v * g.plane + at] = A[v * ncell + c];
      if (nsteps > 0) w_prev[v * g.plane + at] = B[v * ncell + c];
    }
  }
  if (tid == 0 && nsteps > 0) {
    s->cur_sx = sx;
    s->cur_sy = sy;
    s->dt = dt;
    if (log) s->nstep = n;
    if (st) atomicOr(&s->status, st);
  }
}

template <class M>
void* resident_fn(int bc) {
  if (bc == kPeriodic) return reinterpret_cast<void*>(&resident_run_kernel<M, kPeriodic>);
  if (bc == kTransmissive) return reinterpret_cast<void*>(&resident_run_kernel<M, kTransmissive>);
  if (bc == kDirichlet) return reinterpret_cast<void*>(&resident_run_kernel<M, kDirichlet>);
  return nullptr;
}

}  // namespace

// nsteps adaptive steps of the grid of `a` (a.win: the current state) in one
// workgroup: the final state goes to w_last, the one before it to w_prev.
// model: 0 advection, 1 Euler, 2 spray (lognormal closure).
hipError_t launch_resident_run(const StepArgs& a, int model, double* w_last, double* w_prev,
                               int nsteps, hipStream_t st) {
  void* f = nullptr;
  if (model == 0) f = resident_fn<Adv>(a.g.bc);
  else if (model == 1) f = resident_fn<Euler>(a.g.bc);
  else if (model == 2) f = resident_fn<Spray>(a.g.bc);
  const int nv = model == 0 ? 1 : (model == 1 ? 4 : 6);
  if (!f || nsteps < 0 ||
      2LL * nv * a.g.nx * a.g.ny > static_cast<long long>(kResidentDoubles))
    return hipErrorInvalidValue;
  StepArgs copy = a;
  void* args[] = {&copy, &w_last, &w_prev, &nsteps};
  const int threads = model == 0 ? res::threads<Adv>() : res::threads<Euler>();
  return hipLaunchKernel(f, dim3(1), dim3(threads), args, 0, st);
}

}  // namespace fvm
