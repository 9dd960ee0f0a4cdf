// fvm_step.hpp -- device building blocks of the fused step, shared by the
// single-grid kernel and the persistent batched kernel: boundary index maps,
// the marching wave strip, the NaN-propagating speed reduction and the
// device-side time step.
#pragma once

#include <hip/hip_runtime.h>

#include <cfloat>
#include <cstdint>

#include "fvm_internal.hpp"
#include "fvm_models.hpp"

// Launch bounds of the marching kernels: WPB waves per workgroup and, when
// FVM_MIN_WAVES > 0, at least that many waves per SIMD (which caps the
// registers the compiler may use per lane).
#ifndef FVM_MIN_WAVES
#define FVM_MIN_WAVES 0
#endif
#if FVM_MIN_WAVES > 0
#define FVM_STEP_BOUNDS(WPB) __launch_bounds__((WPB) * 64, FVM_MIN_WAVES)
#else
#define FVM_STEP_BOUNDS(WPB) __launch_bounds__((WPB) * 64)
#endif

namespace fvm {

// ---- index helpers -------------------------------------------------------------

// column of lane (may be -1 or >= nx): periodic wrap, transmissive clamp; any
// further lane (past the grid) is clamped into range, its result is unused.
template <int BC>
__device__ __forceinline__ int col_index(int i, int nx) {
  int c;
  if (BC == 0) {
    c = i < 0 ? i + nx : (i >= nx ? i - nx : i);
  } else {
    c = i;
  }
  c = c < 0 ? 0 : c;
  return c >= nx ? nx - 1 : c;
}

// row r in [-1, ny]
template <int BC>
__device__ __forceinline__ int row_index(int r, int ny) {
  if (BC == 0) return r < 0 ? ny - 1 : (r >= ny ? 0 : r);
  return r < 0 ? 0 : (r >= ny ? ny - 1 : r);
}

template <int NV, int BC>
__device__ __forceinline__ void load_row(double* w, const double* __restrict__ base,
                                         const GridGeom& g, int r) {
  const size_t off = static_cast<size_t>(row_index<BC>(r, g.ny)) * g.ld;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
#if FVM_NT_LOADS
    w[v] = __builtin_nontemporal_load(base + v * g.plane + off);
#else
    w[v] = base[v * g.plane + off];
#endif
  }
}

__device__ __forceinline__ unsigned long long bits(double x) {
  return static_cast<unsigned long long>(__double_as_longlong(x));
}
__device__ __forceinline__ unsigned long long umax64(unsigned long long a, unsigned long long b) {
  return a > b ? a : b;
}

__device__ __forceinline__ unsigned long long wave_max64(unsigned long long x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long y = __shfl_xor(x, o, 64);
    x = umax64(x, y);
  }
  return x;
}

// ---- one strip ---------------------------------------------------------------
// Updates rows [j0, j1) of columns [xs, xs+62) ∩ [0, nx) and folds the new
// cells' speeds into (bx, by).
template <class M, int BC>
__device__ __forceinline__ void march_strip(const M& m, const double* __restrict__ win,
                                            double* __restrict__ wout,
                                            const double* __restrict__ ug, const GridGeom& g,
                                            int xs, int j0, int j1, double mux, double muy,
                                            double dt, unsigned long long& bx,
                                            unsigned long long& by) {
  constexpr int NV = M::NV;
  using Prim = typename M::Prim;
  const int lane = threadIdx.x & (kWave - 1);
  const int i = xs - 1 + lane;
  const int ic = col_index<BC>(i, g.nx);
  const bool out = (lane >= 1) & (lane <= kOutPerWave) & (i < g.nx);
  const double* base = win + ic;

  // Register ring of R = PF + 2 rows: while row j is updated, rows j+1 ..
  // j+PF are loaded or in flight and the load of row j+1+PF is issued into
  // the slot that held row j-1. Slot of row r: (r - j0) mod R (row j0-1 ->
  // slot R-1). The loop is unrolled R times so every slot is a fixed set of
  // registers and no row is ever copied. The primitives and the y-face flux
  // below each row live in rings of the same period.
  constexpr int PF = M::kPrefetch;
  constexpr int R = PF + 2;
  double W[R][NV], G[R][NV];
  Prim P[R];
  // Rows past the strip's last halo row j1 are never needed: their loads
  // re-read row j1 (an L2 hit) and the rows computed past j1 - 1 are not
  // stored, so the unrolled body carries no branches.
  load_row<NV, BC>(W[R - 1], base, g, j0 - 1);
  load_row<NV, BC>(W[0], base, g, j0);
#pragma unroll
  for (int p = 1; p <= PF; ++p) load_row<NV, BC>(W[p], base, g, min(j0 + p, j1));
  m.prim(W[R - 1], P[R - 1]);
  m.prim(W[0], P[0]);
  m.template flux<1>(W[R - 1], P[R - 1], W[0], P[0], G[0]);

  for (int jb = j0; jb < j1; jb += R) {
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int j = jb + u;
      {
        const int c = u, n = (u + 1) % R, l = (u + R - 1) % R;
        load_row<NV, BC>(W[l], base, g, min(j + 1 + PF, j1));
        m.prim(W[n], P[n]);
        double Fe[NV], Wr[NV], Wo[NV];
        Prim Pr;
        m.template flux<1>(W[c], P[c], W[n], P[n], G[n]);
        m.shift_next(W[c], P[c], Wr, Pr);
        m.template flux<0>(W[c], P[c], Wr, Pr, Fe);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const double Fw = from_prev(Fe[v]);
          Wo[v] = W[c][v] - fma(mux, Fe[v] - Fw, muy * (G[n][v] - G[c][v]));
        }
        const size_t cell = static_cast<size_t>(j) * g.ld + ic;
        if constexpr (NV == 6) {
          m.source(Wo, ug[cell], ug[g.plane + cell], dt);
        }
        if (out && j < j1) {
#pragma unroll
          for (int v = 0; v < NV; ++v)
            __builtin_nontemporal_store(Wo[v], wout + v * g.plane + cell);
          double sx, sy;
          m.speeds(Wo, sx, sy);
          bx = umax64(bx, bits(sx));
          by = umax64(by, bits(sy));
        }
      }
#if FVM_SCHED_BARRIER
      // keep the scheduler from interleaving consecutive rows, which would
      // lengthen live ranges and cost occupancy
      __builtin_amdgcn_sched_barrier(0);
#endif
    }
  }
}

// ---- reductions and the device-side time step ------------------------------------

// Adaptive dt from the maxima: dt = C / (Sx/dx + Sy/dy); dt_max if both are 0.
__device__ __forceinline__ double next_dt(const GridGeom& g, double sx, double sy) {
  if (sx == 0.0 && sy == 0.0) return g.dt_max;
  return g.cfl / (sx / g.dx + sy / g.dy);
}

// Called by the last workgroup of a launch: reads and clears the maxima,
// records the current state's maxima and the next dt, logs the dt used.
__device__ inline void finalize_grid(GridScratch* s, const GridGeom& g, double dt_used,
                                     double* dt_log, int cap, int stride, double* dt_out) {
  const double sx = __longlong_as_double(static_cast<long long>(atomicExch(&s->smax[0], 0ull)));
  const double sy = __longlong_as_double(static_cast<long long>(atomicExch(&s->smax[1], 0ull)));
  unsigned int st = 0;
  if (!(sx <= DBL_MAX) || !(sy <= DBL_MAX)) st |= kStatusNonFinite;
  const double dtn = next_dt(g, sx, sy);
  if (!(dtn > 0.0)) st |= kStatusDt;
  s->cur_sx = sx;
  s->cur_sy = sy;
  s->dt = dtn;
  if (st) atomicOr(&s->status, st);
  if (dt_log) {
    const unsigned int n = s->nstep;
    if (n < static_cast<unsigned int>(cap)) dt_log[static_cast<size_t>(n) * stride] = dt_used;
    s->nstep = n + 1;
  }
  if (dt_out) *dt_out = dtn;
  __threadfence();
  atomicExch(&s->arrive, 0u);
}

// Workgroup max of (bx, by); thread 0 commits it and returns true if its
// workgroup is the last of `total` arrivals on s.
template <int WPB>
__device__ __forceinline__ bool block_commit(unsigned long long bx, unsigned long long by,
                                             GridScratch* s, unsigned int total) {
  __shared__ unsigned long long red[2][WPB];
  __shared__ bool last;
  bx = wave_max64(bx);
  by = wave_max64(by);
  const int wave = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) {
    red[0][wave] = bx;
    red[1][wave] = by;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long mx = red[0][0], my = red[1][0];
#pragma unroll
    for (int k = 1; k < WPB; ++k) {
      mx = umax64(mx, red[0][k]);
      my = umax64(my, red[1][k]);
    }
    atomicMax(&s->smax[0], mx);
    atomicMax(&s->smax[1], my);
    __threadfence();
    const unsigned int t = atomicAdd(&s->arrive, 1u);
    last = (t == total - 1);
  }
  __syncthreads();
  return last;
}

// dt of this launch, and for a fixed-dt step the paper's check
// dt * max(Sx, Sy) <= min(dx, dy) (a failed check makes the step a copy).
__device__ __forceinline__ double launch_dt(const StepArgs& a, bool& cfl_fail) {
  cfl_fail = false;
  if (a.mode == kDtAdaptive) return a.scr->dt;
  if (a.mode == kDtArray) return a.dts[a.k];
  const double smax = a.scr->cur_sx > a.scr->cur_sy ? a.scr->cur_sx : a.scr->cur_sy;
  cfl_fail = a.dt_arg * smax > a.g.hmin;
  return a.dt_arg;
}

// Workgroup b -> tile: workgroups are dealt round-robin over the 8 XCDs, so
// the tiles are split into 8 contiguous row-major ranges and XCD x walks
// range x; vertically adjacent tiles then share that XCD's L2 for their halo
// rows.
__device__ __forceinline__ int xcd_tile(int b, int ntiles) {
  constexpr int kXcd = 8;
  const int x = b % kXcd, k = b / kXcd;
  const int q = ntiles / kXcd, r = ntiles % kXcd;
  return x * q + (x < r ? x : r) + k;
}

}  // namespace fvm
