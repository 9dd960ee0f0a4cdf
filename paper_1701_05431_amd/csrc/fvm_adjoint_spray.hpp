// fvm_adjoint_spray.hpp -- device code of the spray adjoint
// (fvm_adjoint_spray.hip launches it). No cross-lane operations: the two
// phases of a tile are plain per-thread code around one barrier, so a host
// build can run them thread by thread.
//
// The discrete adjoint of one spray step (Sec. 6.1 eq. Essadki with the
// splitting of Sec. 2.2.2 eq. SourceTerm), with the lognormal closure of the
// source.
//
// The step is W* = W - [mux (F_E - F_W) + muy (G_N - G_S)] with the kinetic
// upwind flux F(W_L, W_R) = W_L (u_L.n)+ + W_R (u_R.n)-, then
// W^{n+1} = W* + dt S(W*). Its adjoint, with dt held fixed, takes lam^{n+1}
// back through the source cell by cell,
//   mu = lam^{n+1} + dt J_S(W*)^T lam^{n+1},
// and then through the transport,
//   lam^n_c = mu_c + mux [J_L(c, E)^T (mu_E - mu_c) + J_R(W, c)^T (mu_c - mu_W)]
//                  + muy [same with N and S].
// mu of a neighbour needs that neighbour's W*, so one cell's adjoint reads
// the state two cells away. A workgroup computes mu once per cell of its
// tile and the ring around it, in LDS, then gathers. Boundary rules as in the forward
// step: a transmissive ghost is a copy of its boundary cell (its share goes
// to that cell), a Dirichlet ghost a constant state (no share flows back).
//
// The flux Jacobians are rank one plus a multiple of the identity, so
// J_L^T d = up d + [u_L > 0] (W_L . d) du_L/dW_L with du/dW nonzero in two
// components only, and J_L depends on the left state alone (J_R on the
// right); no 6 x 6 matrix is formed. The source Jacobian follows
// the closure by hand (the width s^2 is a constant where it is clipped).
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/fvm.h"
#include "fvm_internal.hpp"
#include "fvm_models.hpp"

namespace fvm {
namespace sadj {

constexpr double kVac = 1e-300;  // moments at or below it switch velocity and source off
constexpr double kExpQuarterClip = 1.000000002500000003125;  // exp(1e-8 / 4)

enum { kCell = 0, kCopy = 1, kGhost = 2 };

// Neighbour of the real cell (j, i) on side s (0 west, 1 east, 2 south,
// 3 north): a cell of the grid (wrapped on periodic grids), a copy of (j, i)
// (transmissive ghost) or the side's constant state (Dirichlet ghost).
__device__ __forceinline__ int neighbour(const GridGeom& g, int j, int i, int s, int& jj,
                                         int& ii) {
  ii = i + (s == 0 ? -1 : (s == 1 ? 1 : 0));
  jj = j + (s == 2 ? -1 : (s == 3 ? 1 : 0));
  if (ii >= 0 && ii < g.nx && jj >= 0 && jj < g.ny) return kCell;
  if (g.bc == FVM_PERIODIC) {
    ii = ii < 0 ? g.nx - 1 : (ii >= g.nx ? 0 : ii);
    jj = jj < 0 ? g.ny - 1 : (jj >= g.ny ? 0 : jj);
    return kCell;
  }
  ii = i;
  jj = j;
  return g.bc == FVM_TRANSMISSIVE ? kCopy : kGhost;
}

__device__ __forceinline__ void load6(const double* base, const GridGeom& g, int j, int i,
                                      double* w) {
  const double* p = base + static_cast<size_t>(j) * g.ld + i;
#pragma unroll
  for (int v = 0; v < 6; ++v) w[v] = p[v * g.plane];
}

// 1/m_{2/2} of a state, 0 at or below the vacuum threshold (velocity 0)
__device__ __forceinline__ double inv_m2(const double* w) {
  return w[2] > kVac ? recip(w[2]) : 0.0;
}

// velocity along axis D from the state and its 1/m_{2/2}
template <int D>
__device__ __forceinline__ double vel(const double* w, double r) {
  return r != 0.0 ? w[4 + D] * r : 0.0;
}

template <int D>
__device__ __forceinline__ void flux(const double* wl, double rl, const double* wr, double rr,
                                     double* f) {
  const double ul = vel<D>(wl, rl), ur = vel<D>(wr, rr);
  const double up = ul > 0.0 ? ul : 0.0;
  const double um = ur < 0.0 ? ur : 0.0;
#pragma unroll
  for (int k = 0; k < 6; ++k) f[k] = fma(wl[k], up, wr[k] * um);
}

// out += c * J_L(wl, .)^T d along axis D (the left state's Jacobian; r = 1/m_{2/2})
template <int D>
__device__ __forceinline__ void add_jl(const double* wl, double r, const double* d, double c,
                                       double* out) {
  const double u = vel<D>(wl, r);
  if (!(u > 0.0)) return;
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < 6; ++k) s = fma(wl[k], d[k], s);
#pragma unroll
  for (int k = 0; k < 6; ++k) out[k] = fma(c, u * d[k], out[k]);
  out[2] = fma(c, s * (-u * r), out[2]);
  out[4 + D] = fma(c, s * r, out[4 + D]);
}

// out += c * J_R(., wr)^T d along axis D (the right state's Jacobian)
template <int D>
__device__ __forceinline__ void add_jr(const double* wr, double r, const double* d, double c,
                                       double* out) {
  const double u = vel<D>(wr, r);
  if (!(u < 0.0)) return;
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < 6; ++k) s = fma(wr[k], d[k], s);
#pragma unroll
  for (int k = 0; k < 6; ++k) out[k] = fma(c, u * d[k], out[k]);
  out[2] = fma(c, s * (-u * r), out[2]);
  out[4 + D] = fma(c, s * r, out[4 + D]);
}

// index modulo n (n >= 1) for periodic wraps; the offsets stay within a
// tile and its ring of the grid, so one step is the rule and several happen
// only on grids narrower than the ring (no integer division)
__device__ __forceinline__ int wrap(int i, int n) {
  while (i < 0) i += n;
  while (i >= n) i -= n;
  return i;
}

struct SprayAdj {
  const AdjointArgs& a;
  const double* ug;  // gas velocity, 2 planes (uplane, uld)
  double dt, mux, muy;

  // g = J_S(W*)^T lam without the closure's part: the drag rows and the
  // evaporation rows of m_{2/2}, m_{3/2} and q (zero where the source is off)
  __device__ __forceinline__ static void source_rows(const double* ws, const double* lam,
                                                     const double* ugc, double K, double it,
                                                     double r2, double* g) {
#pragma unroll
    for (int v = 0; v < 6; ++v) g[v] = 0.0;
    const double m0 = ws[0];
    // momentum rows: S_{4+d} = m_0 (-K u_d + (ug_d - u_d)/theta), u_d = q_d / m_{2/2}
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      const double ud = ws[4 + d] * r2;
      const double ld = lam[4 + d];
      g[0] = fma(ld, fma(-K, ud, (ugc[d] - ud) * it), g[0]);
      g[2] = fma(ld, m0 * (K + it) * ud * r2, g[2]);
      g[4 + d] = -ld * m0 * (K + it) * r2;
    }
    g[0] = fma(-K, lam[2], g[0]);
    g[1] = -1.5 * K * lam[3];
  }

  // mu = lam + dt J_S(W*)^T lam at a real cell, given its W* (ws), lam
  // (lam) and gas velocity (ugc), with the lognormal closure
  __device__ __forceinline__ void mu_at(const double* ws, const double* lam, const double* ugc,
                                        double* mu) const {
#pragma unroll
    for (int v = 0; v < 6; ++v) mu[v] = lam[v];
    const double m0 = ws[0], m1 = ws[1], m2 = ws[2];
    if (!(m0 > kVac) || !(m1 > kVac) || !(m2 > kVac)) return;
    const double K = a.m.K, it = a.m.inv_theta;
    const double r2 = recip(m2);
    const double l0 = lam[0], l1 = lam[1];
    double g[6];
    source_rows(ws, lam, ugc, K, it, r2, g);
    if (K != 0.0) {
      // the closure rows: S_0 = -K n(S_eps), S_1 = -K/2 m_{-1/2}
      const double r0 = recip(m0), r1 = recip(m1);
      const double L1 = logd(m1 * r0), L2 = logd(m2 * r0);
      double s2 = 4.0 * fma(-2.0, L1, L2);
      const bool clipped = s2 < 1e-8;
      s2 = clipped ? 1e-8 : s2;
      const double mu_ = fma(2.0, L1, -0.25 * s2);
      // m_{-1/2} = m_0 exp(s^2/8 - mu/2) = m_0 q exp(s^2/4), q = m_0 / m_{1/2}:
      // m_{2/2} q^3 with the fitted width, m_0 q e^{1/4e-8} with the clipped
      // one; n(S_eps) with 1/S_eps folded into its exponential
      const double q = m0 * r1;
      const double mmh = clipped ? m0 * q * kExpQuarterClip : m2 * (q * q * q);
      const double z = a.m.log_s_eps - mu_;
      const double rs = rroot(6.283185307179586 * s2);
      const double is2 = 6.283185307179586 * (rs * rs);
      const double n0 = m0 * rs * exp(fma(-(z * z), 0.5 * is2, -a.m.log_s_eps));
      // d ln n(S_eps) = d ln m_0 - ds2 / (2 s^2) + z dmu / s^2 + z^2 ds2 / (2 s^4)
      const double c1 = 0.5 * fma(z * z, is2, -1.0);
      const double dL1[3] = {-r0, r1, 0.0};
      const double dL2[3] = {-r0, 0.0, r2};
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        const double ds2 = clipped ? 0.0 : 4.0 * fma(-2.0, dL1[l], dL2[l]);
        const double dmu = fma(2.0, dL1[l], -0.25 * ds2);
        const double dm0 = l == 0 ? r0 : 0.0;
        const double dlm = fma(-0.5, dmu, fma(0.125, ds2, dm0));
        const double dln = fma(is2, fma(z, dmu, ds2 * c1), dm0);
        g[l] = fma(l1, -0.5 * K * mmh * dlm, g[l]);
        g[l] = fma(l0, -K * n0 * dln, g[l]);
      }
    }
#pragma unroll
    for (int v = 0; v < 6; ++v) mu[v] = fma(dt, g[v], mu[v]);
  }

  // lam^n of the real cell (j, i) from its state c (with r = 1/m_{2/2}), its
  // own mu (mc) and its neighbours' (nb_mu(side, m) fills mu of the
  // neighbour cell on that side)
  template <class NbMu>
  __device__ __forceinline__ void gather(int j, int i, const double* c, double r,
                                         const double* mc, NbMu&& nb_mu, double* out) const {
#pragma unroll
    for (int v = 0; v < 6; ++v) out[v] = mc[v];
    double m[6], d[6];
    int jj, ii;
    // x faces: east (c left of it), west (c right of it)
    // on periodic grids every neighbour is a cell (uniform across the workgroup)
    const bool per = a.g.bc == FVM_PERIODIC;
    int k = per ? kCell : neighbour(a.g, j, i, 1, jj, ii);
    if (k == kCell) {
      nb_mu(1, m);
#pragma unroll
      for (int v = 0; v < 6; ++v) d[v] = m[v] - mc[v];
      add_jl<0>(c, r, d, mux, out);
    } else {
#pragma unroll
      for (int v = 0; v < 6; ++v) d[v] = -mc[v];
      add_jl<0>(c, r, d, mux, out);
      if (k == kCopy) add_jr<0>(c, r, d, mux, out);
    }
    k = per ? kCell : neighbour(a.g, j, i, 0, jj, ii);
    if (k == kCell) {
      nb_mu(0, m);
#pragma unroll
      for (int v = 0; v < 6; ++v) d[v] = mc[v] - m[v];
      add_jr<0>(c, r, d, mux, out);
    } else {
      if (k == kCopy) add_jl<0>(c, r, mc, mux, out);
      add_jr<0>(c, r, mc, mux, out);
    }
    // y faces: north, south
    k = per ? kCell : neighbour(a.g, j, i, 3, jj, ii);
    if (k == kCell) {
      nb_mu(3, m);
#pragma unroll
      for (int v = 0; v < 6; ++v) d[v] = m[v] - mc[v];
      add_jl<1>(c, r, d, muy, out);
    } else {
#pragma unroll
      for (int v = 0; v < 6; ++v) d[v] = -mc[v];
      add_jl<1>(c, r, d, muy, out);
      if (k == kCopy) add_jr<1>(c, r, d, muy, out);
    }
    k = per ? kCell : neighbour(a.g, j, i, 2, jj, ii);
    if (k == kCell) {
      nb_mu(2, m);
#pragma unroll
      for (int v = 0; v < 6; ++v) d[v] = mc[v] - m[v];
      add_jr<1>(c, r, d, muy, out);
    } else {
      if (k == kCopy) add_jl<1>(c, r, mc, muy, out);
      add_jr<1>(c, r, mc, muy, out);
    }
  }
};

// ---- tiles ------------------------------------------------------------------
//
// A workgroup of kTileThreads threads owns kTX x kTY cells, in three phases
// separated by barriers, all from LDS after the first:
//   1. the states of the tile and of the two-cell ring around it (the box),
//      each loaded from HBM once, with 1/m_{2/2} (0 in vacuum) beside them,
//      and (into registers) lam and u_g of the cells that phase 2 needs;
//   2. mu of every cell of the tile and of the one-cell ring, its W* from the
//      box (the ring wraps on periodic grids; outside other grids it is not
//      needed: those faces use the ghost rules);
//   3. lam^n of the tile's cells from mu and their own states.
// Every W*, mu and lam^n is computed as the per-cell formula does, so the
// result does not depend on the tiling. Box cells outside a non-periodic
// grid are not loaded: the ghost rules never read them.

#ifndef FVM_SADJ_THREADS
#define FVM_SADJ_THREADS 512
#endif
// 30 x 14 cells: the mu box (32 x 16) is one value per thread, so no wave
// takes a second mu pass while the others wait at the barrier (3 % faster
// than 64 x 8, whose 66 x 10 mu box is 1.29 per thread)
#ifndef FVM_SADJ_COLS
#define FVM_SADJ_COLS 30
#endif
#ifndef FVM_SADJ_ROWS
#define FVM_SADJ_ROWS 14
#endif

constexpr int kTileThreads = FVM_SADJ_THREADS;
constexpr int kTX = FVM_SADJ_COLS;
constexpr int kTY = FVM_SADJ_ROWS;
constexpr int kBX = kTX + 4, kBY = kTY + 4;  // state box: the tile and a two-cell ring
constexpr int kBox = kBX * kBY;
constexpr int kBoxVars = 7;                  // W and 1/m_{2/2}
constexpr int kRX = kTX + 2, kRY = kTY + 2;  // mu box: the tile and a one-cell ring
constexpr int kRing = kRX * kRY;             // mu values per variable in LDS
constexpr int kLdsDoubles = kBoxVars * kBox + 6 * kRing;

__device__ __forceinline__ SprayAdj make_adj(const AdjointArgs& a, const double* ug) {
  SprayAdj s{a, ug, 0.0, 0.0, 0.0};
  s.dt = a.dts ? a.dts[a.k] : a.dt_arg;
  s.mux = s.dt / a.g.dx;
  s.muy = s.dt / a.g.dy;
  return s;
}

// phase 1: the state box into box[v * kBox + r * kBX + c], v = 6: 1/m_{2/2}
__device__ __forceinline__ void tile_load(const SprayAdj& s, int j0, int i0, int tid,
                                          double* box) {
  const GridGeom& g = s.a.g;
  const bool per = g.bc == FVM_PERIODIC;
  for (int idx = tid; idx < kBox; idx += kTileThreads) {
    const int r = idx / kBX, c = idx % kBX;
    int j = j0 - 2 + r, i = i0 - 2 + c;
    const bool inside = j >= 0 && j < g.ny && i >= 0 && i < g.nx;
    double w[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (inside || per) {
      j = wrap(j, g.ny);
      i = wrap(i, g.nx);
      load6(s.a.w, g, j, i, w);
    }
#pragma unroll
    for (int v = 0; v < 6; ++v) box[v * kBox + idx] = w[v];
    box[6 * kBox + idx] = inv_m2(w);
  }
}

// The real cell of mu-box entry idx (the tile and its one-cell ring),
// wrapped on periodic grids; false where no mu is needed there (outside a
// non-periodic grid, or past the grid's far edge by more than one cell).
__device__ __forceinline__ bool ring_cell(const GridGeom& g, int j0, int i0, int idx, int& j,
                                          int& i) {
  const int r = idx / kRX, c = idx % kRX;
  j = j0 - 1 + r;
  i = i0 - 1 + c;
  bool need = j >= -1 && j <= g.ny && i >= -1 && i <= g.nx;
  if (j < 0 || j >= g.ny || i < 0 || i >= g.nx) {
    need = need && g.bc == FVM_PERIODIC;
    j = wrap(j, g.ny);
    i = wrap(i, g.nx);
  }
  return need;
}

// mu entries per thread, and what each needs from HBM besides the box:
// lam (6) and the gas velocity (2)
constexpr int kMuPasses = (kRing + kTileThreads - 1) / kTileThreads;
constexpr int kPre = 8;

// phase 1 (issued with the box loads): lam and u_g of this thread's mu
// entries into pre[p * kPre + ...] (registers on the GPU)
__device__ __forceinline__ void tile_prefetch(const SprayAdj& s, int j0, int i0, int tid,
                                              double* pre) {
  const GridGeom& g = s.a.g;
#pragma unroll
  for (int p = 0; p < kMuPasses; ++p) {
    const int idx = tid + p * kTileThreads;
    int j, i;
    double* q = pre + p * kPre;
    if (idx < kRing && ring_cell(g, j0, i0, idx, j, i)) {
      load6(s.a.lam_in, g, j, i, q);
      const size_t u0 = static_cast<size_t>(j) * g.uld + i;
      q[6] = s.ug[u0];
      q[7] = s.ug[g.uplane + u0];
    } else {
#pragma unroll
      for (int v = 0; v < kPre; ++v) q[v] = 0.0;
    }
  }
}

// phase 2: mu of the tile and its ring into mu_s[v * kRing + r * kRX + c];
// without SRC (the transport's adjoint alone) mu is the prefetched lam
template <bool SRC = true>
__device__ __forceinline__ void tile_mu(const SprayAdj& s, int j0, int i0, int tid,
                                        const double* box, const double* pre, double* mu_s) {
  const GridGeom& g = s.a.g;
#pragma unroll
  for (int p = 0; p < kMuPasses; ++p) {
    const int idx = tid + p * kTileThreads;
    if (idx >= kRing) break;
    const int r = idx / kRX, c = idx % kRX;
    int j, i;
    double m[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (!SRC) {
#pragma unroll
      for (int v = 0; v < 6; ++v) m[v] = pre[p * kPre + v];
    } else if (ring_cell(g, j0, i0, idx, j, i)) {
      // W* of the real cell (j, i): box position (r + 1, c + 1) and its four
      // neighbours there, or a ghost for a side outside a non-periodic grid
      const int at = (r + 1) * kBX + c + 1;
      double w[5][6], rr[5];
      const int off[5] = {0, -1, 1, -kBX, kBX};  // centre, west, east, south, north
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        int jj, ii;
        const int kind =
            q == 0 || g.bc == FVM_PERIODIC ? kCell : neighbour(g, j, i, q - 1, jj, ii);
        const int src = at + (kind == kCell ? off[q] : 0);
        if (kind == kGhost) {
#pragma unroll
          for (int v = 0; v < 6; ++v) w[q][v] = s.a.ghost[(q - 1) * kMaxVar + v];
          rr[q] = inv_m2(w[q]);
        } else {
#pragma unroll
          for (int v = 0; v < 6; ++v) w[q][v] = box[v * kBox + src];
          rr[q] = box[6 * kBox + src];
        }
      }
      double fe[6], fw[6], gn[6], gs[6], ws[6];
      flux<0>(w[0], rr[0], w[2], rr[2], fe);
      flux<0>(w[1], rr[1], w[0], rr[0], fw);
      flux<1>(w[0], rr[0], w[4], rr[4], gn);
      flux<1>(w[3], rr[3], w[0], rr[0], gs);
#pragma unroll
      for (int v = 0; v < 6; ++v)
        ws[v] = w[0][v] - (s.mux * (fe[v] - fw[v]) + s.muy * (gn[v] - gs[v]));
      s.mu_at(ws, pre + p * kPre, pre + p * kPre + 6, m);
    }
#pragma unroll
    for (int v = 0; v < 6; ++v) mu_s[v * kRing + idx] = m[v];
  }
}

// phase 3: lam^n of the tile's cells from mu_s and the box
__device__ __forceinline__ void tile_out(const SprayAdj& s, int j0, int i0, int tid,
                                         const double* box, const double* mu_s) {
  const GridGeom& g = s.a.g;
  for (int idx = tid; idx < kTX * kTY; idx += kTileThreads) {
    const int rr = idx / kTX, c = idx % kTX;
    const int j = j0 + rr, i = i0 + c;
    if (j >= g.ny || i >= g.nx) continue;
    const int at = (rr + 1) * kRX + c + 1;
    const int bat = (rr + 2) * kBX + c + 2;
    double mc[6], w[6], out[6];
#pragma unroll
    for (int v = 0; v < 6; ++v) {
      mc[v] = mu_s[v * kRing + at];
      w[v] = box[v * kBox + bat];
    }
    const double r = box[6 * kBox + bat];
    auto nb_mu = [mu_s, at](int side, double* m) {
      const int o = side == 0 ? -1 : (side == 1 ? 1 : (side == 2 ? -kRX : kRX));
#pragma unroll
      for (int v = 0; v < 6; ++v) m[v] = mu_s[v * kRing + at + o];
    };
    s.gather(j, i, w, r, mc, nb_mu, out);
    double* p = s.a.lam_out + static_cast<size_t>(j) * g.ld + i;
#pragma unroll
    for (int v = 0; v < 6; ++v) p[v * g.plane] = out[v];
  }
}

}  // namespace sadj
}  // namespace fvm
