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

namespace fvm {
namespace sadj {

constexpr double kVac = 1e-300;  // moments at or below it switch velocity and source off

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

// velocity along axis D and 1/m_{2/2} (0, 0 below the vacuum threshold)
template <int D>
__device__ __forceinline__ double vel(const double* w, double& r) {
  const bool ok = w[2] > kVac;
  r = ok ? 1.0 / w[2] : 0.0;
  return ok ? w[4 + D] * r : 0.0;
}

template <int D>
__device__ __forceinline__ void flux(const double* wl, const double* wr, double* f) {
  double rl, rr;
  const double ul = vel<D>(wl, rl), ur = vel<D>(wr, rr);
  const double up = ul > 0.0 ? ul : 0.0;
  const double um = ur < 0.0 ? ur : 0.0;
#pragma unroll
  for (int k = 0; k < 6; ++k) f[k] = fma(wl[k], up, wr[k] * um);
}

// out += c * J_L(wl, .)^T d along axis D (the left state's Jacobian)
template <int D>
__device__ __forceinline__ void add_jl(const double* wl, const double* d, double c,
                                       double* out) {
  double r;
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
__device__ __forceinline__ void add_jr(const double* wr, const double* d, double c,
                                       double* out) {
  double r;
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

struct SprayAdj {
  const AdjointArgs& a;
  const double* ug;  // gas velocity, 2 planes (uplane, uld)
  double dt, mux, muy;

  __device__ __forceinline__ void state(int kind, int s, int jj, int ii, double* w) const {
    if (kind == kGhost) {
#pragma unroll
      for (int v = 0; v < 6; ++v) w[v] = a.ghost[s * kMaxVar + v];
    } else {
      load6(a.w, a.g, jj, ii, w);
    }
  }

  // W* of the real cell (j, i)
  __device__ __forceinline__ void wstar(int j, int i, double* ws) const {
    double c[6], nw[6], ne[6], ns[6], nn[6];
    load6(a.w, a.g, j, i, c);
    int jj, ii, k;
    k = neighbour(a.g, j, i, 0, jj, ii);
    state(k, 0, jj, ii, nw);
    k = neighbour(a.g, j, i, 1, jj, ii);
    state(k, 1, jj, ii, ne);
    k = neighbour(a.g, j, i, 2, jj, ii);
    state(k, 2, jj, ii, ns);
    k = neighbour(a.g, j, i, 3, jj, ii);
    state(k, 3, jj, ii, nn);
    double fe[6], fw[6], gn[6], gs[6];
    flux<0>(c, ne, fe);
    flux<0>(nw, c, fw);
    flux<1>(c, nn, gn);
    flux<1>(ns, c, gs);
#pragma unroll
    for (int v = 0; v < 6; ++v) ws[v] = c[v] - (mux * (fe[v] - fw[v]) + muy * (gn[v] - gs[v]));
  }

  // mu = lam + dt J_S(W*)^T lam at the real cell (j, i)
  __device__ __forceinline__ void mu_at(int j, int i, double* mu) const {
    double ws[6];
    wstar(j, i, ws);
    load6(a.lam_in, a.g, j, i, mu);
    const double m0 = ws[0], m1 = ws[1], m2 = ws[2];
    if (!(m0 > kVac) || !(m1 > kVac) || !(m2 > kVac)) return;
    const size_t u0 = static_cast<size_t>(j) * a.g.uld + i;
    const double ugc[2] = {ug[u0], ug[a.g.uplane + u0]};
    const double K = a.m.K, it = a.m.inv_theta;
    const double r2 = 1.0 / m2;
    const double l0 = mu[0], l1 = mu[1], l2 = mu[2], l3 = mu[3], l4 = mu[4], l5 = mu[5];
    double g[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    // momentum rows: S_{4+d} = m_0 (-K u_d + (ug_d - u_d)/theta), u_d = q_d / m_{2/2}
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      const double ud = ws[4 + d] * r2;
      const double ld = d == 0 ? l4 : l5;
      g[0] = fma(ld, fma(-K, ud, (ugc[d] - ud) * it), g[0]);
      g[2] = fma(ld, m0 * (K + it) * ud * r2, g[2]);
      g[4 + d] = -ld * m0 * (K + it) * r2;
    }
    g[0] = fma(-K, l2, g[0]);
    g[1] = -1.5 * K * l3;
    if (K != 0.0) {
      // the closure rows: S_0 = -K n(S_eps), S_1 = -K/2 m_{-1/2}
      const double r0 = 1.0 / m0, r1 = 1.0 / m1;
      const double L1 = log(m1 * r0), L2 = log(m2 * r0);
      double s2 = 4.0 * fma(-2.0, L1, L2);
      const bool clipped = s2 < 1e-8;
      s2 = clipped ? 1e-8 : s2;
      const double mu_ = fma(2.0, L1, -0.25 * s2);
      const double mmh = m0 * exp(fma(-0.5, mu_, 0.125 * s2));
      const double z = a.m.log_s_eps - mu_;
      const double n0 =
          m0 / (a.m.s_eps * sqrt(6.283185307179586 * s2)) * exp(-(z * z) / (2.0 * s2));
      const double is2 = 1.0 / s2;
      const double dL1[3] = {-r0, r1, 0.0};
      const double dL2[3] = {-r0, 0.0, r2};
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        const double ds2 = clipped ? 0.0 : 4.0 * fma(-2.0, dL1[l], dL2[l]);
        const double dmu = fma(2.0, dL1[l], -0.25 * ds2);
        const double dm0 = l == 0 ? r0 : 0.0;
        const double dlm = dm0 - 0.5 * dmu + 0.125 * ds2;
        const double dln = dm0 - 0.5 * ds2 * is2 + z * dmu * is2 + 0.5 * z * z * ds2 * is2 * is2;
        g[l] = fma(l1, -0.5 * K * mmh * dlm, g[l]);
        g[l] = fma(l0, -K * n0 * dln, g[l]);
      }
    }
#pragma unroll
    for (int v = 0; v < 6; ++v) mu[v] = fma(dt, g[v], mu[v]);
  }

  // lam^n of the real cell (j, i)
  // lam^n of the real cell (j, i) from its own mu (mc) and its neighbours'
  // (nb_mu(side, m) fills mu of the neighbour cell on that side)
  template <class NbMu>
  __device__ __forceinline__ void gather(int j, int i, const double* mc, NbMu&& nb_mu,
                                         double* out) const {
    double c[6];
    load6(a.w, a.g, j, i, c);
#pragma unroll
    for (int v = 0; v < 6; ++v) out[v] = mc[v];
    double m[6], d[6];
    int jj, ii;
    // x faces: east (c left of it), west (c right of it)
    int k = neighbour(a.g, j, i, 1, jj, ii);
    if (k == kCell) {
      nb_mu(1, m);
#pragma unroll
      for (int v = 0; v < 6; ++v) d[v] = m[v] - mc[v];
      add_jl<0>(c, d, mux, out);
    } else {
#pragma unroll
      for (int v = 0; v < 6; ++v) d[v] = -mc[v];
      add_jl<0>(c, d, mux, out);
      if (k == kCopy) add_jr<0>(c, d, mux, out);
    }
    k = neighbour(a.g, j, i, 0, jj, ii);
    if (k == kCell) {
      nb_mu(0, m);
#pragma unroll
      for (int v = 0; v < 6; ++v) d[v] = mc[v] - m[v];
      add_jr<0>(c, d, mux, out);
    } else {
      if (k == kCopy) add_jl<0>(c, mc, mux, out);
      add_jr<0>(c, mc, mux, out);
    }
    // y faces: north, south
    k = neighbour(a.g, j, i, 3, jj, ii);
    if (k == kCell) {
      nb_mu(3, m);
#pragma unroll
      for (int v = 0; v < 6; ++v) d[v] = m[v] - mc[v];
      add_jl<1>(c, d, muy, out);
    } else {
#pragma unroll
      for (int v = 0; v < 6; ++v) d[v] = -mc[v];
      add_jl<1>(c, d, muy, out);
      if (k == kCopy) add_jr<1>(c, d, muy, out);
    }
    k = neighbour(a.g, j, i, 2, jj, ii);
    if (k == kCell) {
      nb_mu(2, m);
#pragma unroll
      for (int v = 0; v < 6; ++v) d[v] = mc[v] - m[v];
      add_jr<1>(c, d, muy, out);
    } else {
      if (k == kCopy) add_jl<1>(c, mc, muy, out);
      add_jr<1>(c, mc, muy, out);
    }
  }
};

// ---- tiles ------------------------------------------------------------------
//
// A workgroup of kTileThreads threads owns kTX x kTY cells. It first computes
// mu once for every cell of the tile and of the one-cell ring around it (the
// ring wraps on periodic grids; outside other grids it is not needed: those
// faces use the ghost rules) into LDS, then each thread gathers the faces of
// its cells from there. Every mu is computed as the per-cell formula does,
// so the result does not depend on the tiling.

#ifndef FVM_SADJ_THREADS
#define FVM_SADJ_THREADS 512
#endif
#ifndef FVM_SADJ_ROWS
#define FVM_SADJ_ROWS 16
#endif
constexpr int kTileThreads = FVM_SADJ_THREADS;  // a multiple of kTX
constexpr int kTX = 64;                         // one wave across
constexpr int kTY = FVM_SADJ_ROWS;
constexpr int kRX = kTX + 2, kRY = kTY + 2;  // with the ring
constexpr int kRing = kRX * kRY;             // mu values per variable in LDS
static_assert(kTileThreads % kTX == 0, "whole waves across the tile");

__device__ __forceinline__ SprayAdj make_adj(const AdjointArgs& a, const double* ug) {
  SprayAdj s{a, ug, 0.0, 0.0, 0.0};
  s.dt = a.dts ? a.dts[a.k] : a.dt_arg;
  s.mux = s.dt / a.g.dx;
  s.muy = s.dt / a.g.dy;
  return s;
}

// phase 1: mu of the tile and its ring into mu_s[v * kRing + r * kRX + c]
__device__ __forceinline__ void tile_mu(const SprayAdj& s, int j0, int i0, int tid,
                                        double* mu_s) {
  const GridGeom& g = s.a.g;
  for (int idx = tid; idx < kRing; idx += kTileThreads) {
    const int r = idx / kRX, c = idx % kRX;
    int j = j0 - 1 + r, i = i0 - 1 + c;
    bool need = j >= -1 && j <= g.ny && i >= -1 && i <= g.nx;
    if (j < 0 || j >= g.ny || i < 0 || i >= g.nx) {
      need = need && g.bc == FVM_PERIODIC;
      j = j < 0 ? g.ny - 1 : (j >= g.ny ? 0 : j);
      i = i < 0 ? g.nx - 1 : (i >= g.nx ? 0 : i);
    }
    double m[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (need) s.mu_at(j, i, m);
#pragma unroll
    for (int v = 0; v < 6; ++v) mu_s[v * kRing + idx] = m[v];
  }
}

// phase 2: lam^n of the tile's cells from mu_s
__device__ __forceinline__ void tile_out(const SprayAdj& s, int j0, int i0, int tid,
                                         const double* mu_s) {
  const GridGeom& g = s.a.g;
  const int c = tid % kTX;
  for (int rr = tid / kTX; rr < kTY; rr += kTileThreads / kTX) {
    const int j = j0 + rr, i = i0 + c;
    if (j >= g.ny || i >= g.nx) continue;
    const int at = (rr + 1) * kRX + c + 1;
    double mc[6], out[6];
#pragma unroll
    for (int v = 0; v < 6; ++v) mc[v] = mu_s[v * kRing + at];
    auto nb_mu = [mu_s, at](int side, double* m) {
      const int o = side == 0 ? -1 : (side == 1 ? 1 : (side == 2 ? -kRX : kRX));
#pragma unroll
      for (int v = 0; v < 6; ++v) m[v] = mu_s[v * kRing + at + o];
    };
    s.gather(j, i, mc, nb_mu, out);
    double* p = s.a.lam_out + static_cast<size_t>(j) * g.ld + i;
#pragma unroll
    for (int v = 0; v < 6; ++v) p[v * g.plane] = out[v];
  }
}

}  // namespace sadj
}  // namespace fvm
