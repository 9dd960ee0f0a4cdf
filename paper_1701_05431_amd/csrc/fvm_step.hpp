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

// offset of cell (i, j) in the first variable of the spray gas velocity
__device__ __forceinline__ size_t ucell(const GridGeom& g, int j, int i) {
  return static_cast<size_t>(j) * g.uld + i;
}

// Dirichlet boundaries: the prescribed state of one side, for every lane or
// for the lanes where `use` holds.
template <int NV>
__device__ __forceinline__ void ghost_state(double* w, const double* gh, int side) {
#pragma unroll
  for (int v = 0; v < NV; ++v) w[v] = gh[side * kMaxVar + v];
}
template <int NV>
__device__ __forceinline__ void ghost_if(double* w, const double* gh, int side, bool use) {
#pragma unroll
  for (int v = 0; v < NV; ++v) w[v] = use ? gh[side * kMaxVar + v] : w[v];
}

// Row r (-1 or ny) of column c from a halo buffer, if that side has one;
// returns whether it did (r is uniform across the wave, so is the branch).
template <int NV>
__device__ __forceinline__ bool halo_row(double* w, const Halo& h, const GridGeom& g, int r,
                                         int c) {
  const double* src = r < 0 ? h.s : h.n;
  if (!src) return false;
#pragma unroll
  for (int v = 0; v < NV; ++v) w[v] = src[v * g.rld + c];
  return true;
}

// Row r of a strip's column c (base = w + c); r may be -1 or ny (the ghost
// rows). Those rows come from the halo buffers when the side has one, else
// from the boundary rule: with Dirichlet boundaries the south / north states
// (r is uniform across the wave, so are the branches).
template <int NV, int BC>
__device__ __forceinline__ void load_row(double* w, const double* __restrict__ base,
                                         const GridGeom& g, int r,
                                         const double* gh = nullptr, const Halo* h = nullptr,
                                         int c = 0) {
  if (h && (r < 0 || r >= g.ny)) {
    if (halo_row<NV>(w, *h, g, r, c)) return;
  }
  if constexpr (BC == kDirichlet) {
    if (r < 0 || r >= g.ny) {
      ghost_state<NV>(w, gh, r < 0 ? kSouth : kNorth);
      return;
    }
  }
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

// ---- the marching wave strip ----------------------------------------------------------
// A wave strip updates rows [j0, j1) of a band of consecutive columns and
// folds the new cells' speeds into (bx, by). Both lane layouts below keep a
// register ring of R = PF + 2 rows: while row j is updated, rows j+1 .. j+PF
// are loaded or in flight and the load of row j+1+PF goes into the slot that
// held row j-1 (slot of row r: (r - j0) mod R, row j0-1 in slot R-1). The row
// loop is unrolled R times so every slot is a fixed set of registers and no
// row is copied; the primitives and the y-face flux below each row live in
// rings of the same period. Rows past the strip's last halo row j1 are never
// needed: their loads re-read row j1 and the rows computed past j1 - 1 are
// not stored, so the unrolled body carries no branches.

// ---- one cell per lane -------------------------------------------------------------
// Lane l holds cell xs+l: a wave updates 64 consecutive cells (one aligned
// 512-byte segment per variable and row). The left face of lane 0 and the
// right face of lane 63 come from a halo cell (lane 0: column xs-1, lane 63:
// column xs+64) passed through the same flux code, as in the two-cells layout;
// the other x-faces use DPP moves. EDGE strips reach past the grid's last
// column (addresses through the boundary map, stores masked).
template <class M, int BC, bool EDGE, bool HALO = false>
__device__ __forceinline__ void march_strip1(const M& m, const double* __restrict__ win,
                                             double* __restrict__ wout,
                                             const double* __restrict__ ug, const GridGeom& g,
                                             int xs, int j0, int j1, double mux, double muy,
                                             double dt, unsigned long long& bx,
                                             unsigned long long& by,
                                             const double* gh = nullptr, Halo halo = {}) {
  constexpr int NV = M::NV;
  using Prim = typename M::Prim;
  const int lane = threadIdx.x & (kWave - 1);
  const bool first = lane == 0, last = lane == kWave - 1;
  const int x = xs + lane;
  const int cx = EDGE ? col_index<BC>(x, g.nx) : x;
  const bool ok = !EDGE || x < g.nx;
  const int hx = first ? xs - 1 : xs + kWave;  // halo column of lanes 0 and 63
  const int ch = col_index<BC>(hx, g.nx);
  const double* base = win + cx;
  // Dirichlet: the halo column or this lane's column is outside the grid
  const bool h_out = hx < 0 || hx >= g.nx;
  const int h_side = first ? kWest : kEast;
  auto wrow = [&](double* w, int r) {
    load_row<NV, BC>(w, base, g, r, gh, HALO ? &halo : nullptr, cx);
    if constexpr (BC == kDirichlet && EDGE) ghost_if<NV>(w, gh, kEast, x >= g.nx);
  };
  auto hrow = [&](double* w, int r) {
    load_row<NV, BC>(w, win + ch, g, r, gh, HALO ? &halo : nullptr, ch);
    if constexpr (BC == kDirichlet) ghost_if<NV>(w, gh, h_side, h_out);
  };

  constexpr int PF = M::kPrefetch1;
  constexpr int R = PF + 2;
  double W[R][NV], H[R][NV], G[R][NV];
  Prim P[R];
  wrow(W[R - 1], j0 - 1);
  wrow(W[0], j0);
  hrow(H[0], j0);
#pragma unroll
  for (int p = 1; p <= PF; ++p) {
    wrow(W[p], min(j0 + p, j1));
    hrow(H[p], min(j0 + p, j1 - 1));
  }
  m.prim(W[R - 1], P[R - 1]);
  m.prim(W[0], P[0]);
  m.template flux<1>(W[R - 1], P[R - 1], W[0], P[0], G[0]);

  for (int jb = j0; jb < j1; jb += R) {
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int j = jb + u;
      const int c = u, n = (u + 1) % R, l = (u + R - 1) % R;
      wrow(W[l], min(j + 1 + PF, j1));
      hrow(H[l], min(j + 1 + PF, j1 - 1));
      m.prim(W[n], P[n]);
      m.template flux<1>(W[c], P[c], W[n], P[n], G[n]);
      double Fr[NV], Fh[NV], Wr[NV], Fp[NV], Wo[NV];
      Prim Pr, Ph;
      m.prim(H[c], Ph);
      // east face: the next lane's cell, lane 63's halo cell
      m.shift_next(W[c], P[c], Wr, Pr);
#pragma unroll
      for (int v = 0; v < NV; ++v) Wr[v] = last ? H[c][v] : Wr[v];
      Pr = M::pick(last, Ph, Pr);
      m.template flux<0>(W[c], P[c], Wr, Pr, Fr);
      // west face: the previous lane's east face, lane 0's from its halo cell
      // (the cross-lane move runs with every lane active)
      m.template flux<0>(H[c], Ph, W[c], P[c], Fh);
#pragma unroll
      for (int v = 0; v < NV; ++v) Fp[v] = from_prev(Fr[v]);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const double fw = first ? Fh[v] : Fp[v];
        Wo[v] = W[c][v] - fma(mux, Fr[v] - fw, muy * (G[n][v] - G[c][v]));
      }
      const size_t cell = static_cast<size_t>(j) * g.ld + cx;
      if constexpr (M::kSource) {
        // rows past the strip are computed but not stored; keep their
        // gas-velocity reads inside the field
        const size_t uc = ucell(g, min(j, j1 - 1), cx);
        m.source(Wo, ug[uc], ug[g.uplane + uc], dt);
      }
      if (ok && j < j1) {
#pragma unroll
        for (int v = 0; v < NV; ++v)
          __builtin_nontemporal_store(Wo[v], wout + v * g.plane + cell);
        double sx, sy;
        m.speeds(Wo, sx, sy);
        bx = umax64(bx, bits(sx));
        by = umax64(by, bits(sy));
      }
    }
  }
}

// ---- one strip, two cells per lane ------------------------------------------------
// The wide layout: lane l holds cells xs+2l and xs+2l+1, so a wave updates 128
// consecutive cells and every load and store is an aligned 16-byte access
// (row pitch even, buffers 16-byte aligned). The face between a lane's two
// cells is computed in the lane, the face to the next lane's first cell with
// DPP moves, and the two faces at the strip's ends from a halo cell that
// each lane loads (lane 0: column xs-1, lane 63: column xs+128): lane 63 takes
// it as the right cell of its (b | next) face, and every lane evaluates
// (halo | a), which only lane 0 keeps as its west face. EDGE strips
// reach past the grid's last column: there every cell is addressed through
// the boundary map (past-the-end cells hold the ghost values that their left
// neighbour needs) and stores are masked per cell.
typedef double dbl2 __attribute__((ext_vector_type(2)));

template <int NV, int BC, bool EDGE>
__device__ __forceinline__ void load_pair(double* a, double* b, const double* __restrict__ w,
                                          const GridGeom& g, int ca, int cb, int r,
                                          const double* gh = nullptr, bool a_out = false,
                                          bool b_out = false, const Halo* h = nullptr) {
  if (h && (r < 0 || r >= g.ny)) {
    if (halo_row<NV>(a, *h, g, r, ca)) {
      halo_row<NV>(b, *h, g, r, cb);
      return;
    }
  }
  if constexpr (BC == kDirichlet) {
    if (r < 0 || r >= g.ny) {  // uniform
      ghost_state<NV>(a, gh, r < 0 ? kSouth : kNorth);
      ghost_state<NV>(b, gh, r < 0 ? kSouth : kNorth);
      return;
    }
  }
  const size_t off = static_cast<size_t>(row_index<BC>(r, g.ny)) * g.ld;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const double* p = w + v * g.plane + off;
    if (EDGE) {
      a[v] = p[ca];
      b[v] = p[cb];
    } else {
      const dbl2 x = *reinterpret_cast<const dbl2*>(p + ca);
      a[v] = x.x;
      b[v] = x.y;
    }
  }
  if constexpr (BC == kDirichlet && EDGE) {  // columns past the east edge
    ghost_if<NV>(a, gh, kEast, a_out);
    ghost_if<NV>(b, gh, kEast, b_out);
  }
}

template <class M, int BC, bool EDGE, int PF = M::kPrefetch2, bool HALO = false,
          bool DOWN = false>
__device__ __forceinline__ void march_strip2(const M& m, const double* __restrict__ win,
                                             double* __restrict__ wout,
                                             const double* __restrict__ ug, const GridGeom& g,
                                             int xs, int j0, int j1, double mux, double muy,
                                             double dt, unsigned long long& bx,
                                             unsigned long long& by,
                                             const double* gh = nullptr, Halo halo = {}) {
  constexpr int NV = M::NV;
  using Prim = typename M::Prim;
  const int lane = threadIdx.x & (kWave - 1);
  const bool first = lane == 0, last = lane == kWave - 1;
  const int xa = xs + 2 * lane, xb = xa + 1;
  const int ca = EDGE ? col_index<BC>(xa, g.nx) : xa;
  const int cb = EDGE ? col_index<BC>(xb, g.nx) : xb;
  const bool oka = !EDGE || xa < g.nx, okb = !EDGE || xb < g.nx;
  const int hx = first ? xs - 1 : xs + 2 * kWave;  // halo column of lanes 0 and 63
  const int ch = col_index<BC>(hx, g.nx);
  // Dirichlet: the halo column is outside the grid
  const bool h_out = hx < 0 || hx >= g.nx;
  const int h_side = first ? kWest : kEast;
  auto prow = [&](double* a, double* b, int r) {
    load_pair<NV, BC, EDGE>(a, b, win, g, ca, cb, r, gh, !oka, !okb, HALO ? &halo : nullptr);
  };
  auto hrow = [&](double* w, int r) {
    load_row<NV, BC>(w, win + ch, g, r, gh, HALO ? &halo : nullptr, ch);
    if constexpr (BC == kDirichlet) ghost_if<NV>(w, gh, h_side, h_out);
  };

  // Rows march up from j0, or with DOWN from j1 - 1 down (alternate tiles
  // of a column go opposite ways, so vertical neighbours read the rows they
  // share at about the same time and the second read hits L2); the y-face
  // between the current row and the next one in the march is computed with
  // the lower row first either way, so results do not depend on it.
  constexpr int R = PF + 2;  // PF rows of loads in flight
  constexpr int S = DOWN ? -1 : 1;
  const int jf = DOWN ? j1 - 1 : j0;  // the first row of the march
  const int jh = DOWN ? j0 - 1 : j1;  // the halo row past its last
  auto ahead = [&](int r) { return DOWN ? max(r, jh) : min(r, jh); };
  auto ahead_h = [&](int r) { return DOWN ? max(r, j0) : min(r, j1 - 1); };
  // GA[k], GB[k]: the y-face between the rows in slots k and k - 1 of the
  // march (the previous row's)
  double A[R][NV], B[R][NV], H[R][NV], GA[R][NV], GB[R][NV];
  Prim PA[R], PB[R];
  prow(A[R - 1], B[R - 1], jf - S);
  prow(A[0], B[0], jf);
  hrow(H[0], jf);
#pragma unroll
  for (int p = 1; p <= PF; ++p) {
    prow(A[p], B[p], ahead(jf + S * p));
    hrow(H[p], ahead_h(jf + S * p));
  }
  m.prim(A[R - 1], PA[R - 1]);
  m.prim(B[R - 1], PB[R - 1]);
  m.prim(A[0], PA[0]);
  m.prim(B[0], PB[0]);
  {
    const int lo = DOWN ? 0 : R - 1, up = DOWN ? R - 1 : 0;
    m.template flux<1>(A[lo], PA[lo], A[up], PA[up], GA[0]);
    m.template flux<1>(B[lo], PB[lo], B[up], PB[up], GB[0]);
  }

  for (int jb = jf; DOWN ? jb > jh : jb < jh; jb += S * R) {
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int j = jb + S * u;
      const int c = u, n = (u + 1) % R, l = (u + R - 1) % R;
      prow(A[l], B[l], ahead(j + S * (1 + PF)));
      hrow(H[(u + PF + 1) % R], ahead_h(j + S * (1 + PF)));
      m.prim(A[n], PA[n]);
      m.prim(B[n], PB[n]);
      const int glo = DOWN ? n : c, gup = DOWN ? c : n;
      m.template flux<1>(A[glo], PA[glo], A[gup], PA[gup], GA[n]);
      m.template flux<1>(B[glo], PB[glo], B[gup], PB[gup], GB[n]);
      // row j's north and south faces
      const int kn = DOWN ? c : n, ks = DOWN ? n : c;
      double Fab[NV], Fr[NV], Fh[NV], Wr[NV], Oa[NV], Ob[NV];
      Prim Pr, Ph;
      m.template flux<0>(A[c], PA[c], B[c], PB[c], Fab);
      m.prim(H[c], Ph);
      // (b | next lane's a); lane 63's right cell is its halo cell
      m.shift_next(A[c], PA[c], Wr, Pr);
#pragma unroll
      for (int v = 0; v < NV; ++v) Wr[v] = last ? H[c][v] : Wr[v];
      Pr = M::pick(last, Ph, Pr);
      m.template flux<0>(B[c], PB[c], Wr, Pr, Fr);
      // a's west face: the previous lane's (b | a), lane 0's (halo | a); the
      // cross-lane move runs with every lane active (a DPP read from a lane
      // that is switched off yields 0)
      m.template flux<0>(H[c], Ph, A[c], PA[c], Fh);
      double Fp[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) Fp[v] = from_prev(Fr[v]);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const double fw = first ? Fh[v] : Fp[v];
        Oa[v] = A[c][v] - fma(mux, Fab[v] - fw, muy * (GA[kn][v] - GA[ks][v]));
        Ob[v] = B[c][v] - fma(mux, Fr[v] - Fab[v], muy * (GB[kn][v] - GB[ks][v]));
      }
      const size_t row = static_cast<size_t>(j) * g.ld;
      if constexpr (M::kSource) {
        double ua[2], ub[2];
        GridGeom gu = g;
        gu.ld = g.uld;
        gu.plane = g.uplane;
        // rows past the strip read the clamped gas velocity (never stored)
        load_pair<2, BC == kDirichlet ? kTransmissive : BC, EDGE>(ua, ub, ug, gu, ca, cb, j);
        m.source(Oa, ua[0], ua[1], dt);
        m.source(Ob, ub[0], ub[1], dt);
      }
      if (j >= j0 && j < j1) {
        if (EDGE) {
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            if (oka) __builtin_nontemporal_store(Oa[v], wout + v * g.plane + row + ca);
            if (okb) __builtin_nontemporal_store(Ob[v], wout + v * g.plane + row + cb);
          }
        } else {
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            const dbl2 o = {Oa[v], Ob[v]};
            __builtin_nontemporal_store(o, reinterpret_cast<dbl2*>(wout + v * g.plane + row + ca));
          }
        }
        double sx, sy;
        if (oka) {
          m.speeds(Oa, sx, sy);
          bx = umax64(bx, bits(sx));
          by = umax64(by, bits(sy));
        }
        if (okb) {
          m.speeds(Ob, sx, sy);
          bx = umax64(bx, bits(sx));
          by = umax64(by, bits(sy));
        }
      }
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
// records the current state's maxima and the next dt, and for a step
// (log_step) appends the dt used to the run's dt log if it has one.
__device__ inline void finalize_grid(GridScratch* s, const GridGeom& g, double dt_used,
                                     bool log_step, double* dt_out) {
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
  double* const dt_log = s->log;
  if (log_step && dt_log) {
    const unsigned int n = s->nstep;
    if (n < static_cast<unsigned int>(s->log_cap))
      dt_log[static_cast<size_t>(n) * s->log_stride] = dt_used;
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
  if (a.mode == kDtValue) return a.dt_arg;
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
