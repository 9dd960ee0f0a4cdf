// fvm_adjoint.hpp -- discrete adjoint of the transport step (advection, Euler):
// the per-face transposed Jacobians and the wave strips, device side.
//
// For W^{n+1} = W^n - mux (F_{i+1/2} - F_{i-1/2}) - muy (G_{j+1/2} - G_{j-1/2})
// with F_{i+1/2} = F~(W_i, W_{i+1}) (Sec. 2.2.1) and dt held fixed, the
// transpose of the step's Jacobian applied to lambda = lambda^{n+1} is
//   lambda^n_i = lambda_i + mux [J_L(i+1/2)^T (lambda_{i+1} - lambda_i)
//                              + J_R(i-1/2)^T (lambda_i - lambda_{i-1})] + (y),
// J_L = dF~/dW_L = A(W_L)/2 + sigma/2 I - (W_R - W_L) (dsigma/dW_L)^T / 2,
// J_R = dF~/dW_R = A(W_R)/2 - sigma/2 I - (W_R - W_L) (dsigma/dW_R)^T / 2,
// where A = dF.n/dW and sigma = max(s_L, s_R) follows its left argument on
// ties. On a transmissive boundary the ghost cell equals the boundary cell and
// has no update of its own: its multiplier is zero and its sensitivity goes to
// the boundary cell.
//
// The kernel has the forward kernel's shape: a wave strip marches up the rows;
// each face's pair (J_L^T d, J_R^T d), d = lambda_R - lambda_L, is computed
// once, the left cell keeps J_L^T d and the right cell receives J_R^T d (from
// the previous row for y-faces, from the lane on its left for x-faces).
// A^T d is evaluated matrix-free:
//   T = d1 W1 + d2 W2 + d3 (E + p),  Q = d_{1+D} + d3 u_n,
//   (A^T d)_0 = -u_n T / rho + (gamma-1) |u|^2/2 Q
//   (A^T d)_1 = u_n d1 + [D=0] (d0 + T/rho) - (gamma-1) u Q
//   (A^T d)_2 = u_n d2 + [D=1] (d0 + T/rho) - (gamma-1) v Q
//   (A^T d)_3 = u_n d3 + (gamma-1) Q
// and ds/dW for s = |u_n| + c is sign(u_n) du_n/dW + gamma/(2 c rho)
// (dp/dW - p/rho e_0).
#pragma once

#include <hip/hip_runtime.h>

#include "fvm_internal.hpp"
#include "fvm_models.hpp"

// Rows of (W, lambda) loads in flight per adjoint strip, one and two cells
// per lane.
#ifndef FVM_ADJ_PREFETCH
#define FVM_ADJ_PREFETCH 2
#endif
#ifndef FVM_ADJ_PREFETCH2
#define FVM_ADJ_PREFETCH2 1
#endif

namespace fvm {

struct AdjAdv {
  static constexpr int NV = 1;
  static constexpr bool kCellA = false;  // face() returns the whole shares
  struct Prim {};
  double ax, ay;
  __device__ explicit AdjAdv(const ModelConsts& m) : ax(m.ax), ay(m.ay) {}
  __device__ __forceinline__ void prim(const double*, Prim&) const {}
  template <int D>
  __device__ __forceinline__ void face(const double*, const Prim&, const double*, const Prim&,
                                       const double* d, double* a, double* b) const {
    const double s = D == 0 ? ax : ay;
    a[0] = (s > 0.0 ? s : 0.0) * d[0];
    b[0] = (s < 0.0 ? s : 0.0) * d[0];
  }
  __device__ __forceinline__ void shift_next(const double* w, const Prim&, double* wr,
                                             Prim&) const {
    wr[0] = from_next(w[0]);
  }
};

struct AdjEuler {
  static constexpr int NV = 4;
  // face() leaves out the 0.5 A(W)^T d terms; each cell adds 0.5 A(W)^T of
  // the sum of its faces' d (at_d), once per axis
  static constexpr bool kCellA = true;
  struct Prim { double r, u, v, p, c; };
  double gamma, gm1;
  __device__ explicit AdjEuler(const ModelConsts& m) : gamma(m.gamma), gm1(m.gm1) {}
  // (the forward step's refined reciprocal and square root)
  __device__ __forceinline__ void prim(const double* w, Prim& q) const {
    q.r = recip(w[0]);
    q.u = w[1] * q.r;
    q.v = w[2] * q.r;
    q.p = gm1 * fma(-0.5, fma(w[1], q.u, w[2] * q.v), w[3]);
    q.c = root(gamma * q.p * q.r);
  }
  // out = A(W)^T d along axis D (written with fused multiply-adds: the
  // kernel is bound by this arithmetic)
  template <int D>
  __device__ __forceinline__ void at_d(const double* w, const Prim& q, const double* d,
                                       double* out) const {
    const double un = D == 0 ? q.u : q.v;
    const double T = fma(d[1], w[1], fma(d[2], w[2], d[3] * (w[3] + q.p)));
    const double gQ = gm1 * fma(d[3], un, d[1 + D]);
    const double Tr = T * q.r;
    const double hq2 = 0.5 * fma(q.u, q.u, q.v * q.v);
    out[0] = fma(-un, Tr, hq2 * gQ);
    out[1] = fma(-gQ, q.u, un * d[1]);
    out[2] = fma(-gQ, q.v, un * d[2]);
    out[3] = fma(un, d[3], gQ);
    out[1 + D] += d[0] + Tr;
  }
  // ds/dW of s = |u_n| + c
  template <int D>
  __device__ __forceinline__ void dspeed(const Prim& q, double* gs) const {
    const double un = D == 0 ? q.u : q.v;
    const double sr = un >= 0.0 ? q.r : -q.r;  // sign(u_n) / rho
    const double k = 0.5 * gamma * q.r * recip(q.c);
    const double hq2 = 0.5 * fma(q.u, q.u, q.v * q.v);
    const double kg = k * gm1;
    gs[0] = fma(k, fma(gm1, hq2, -q.p * q.r), -sr * un);
    gs[1] = -kg * q.u;
    gs[2] = -kg * q.v;
    gs[3] = kg;
    gs[1 + D] += sr;
  }
  // The Rusanov face F = (F(W_L) + F(W_R))/2 - s (W_R - W_L)/2 with
  // d = lambda_R - lambda_L: a = (dF/dW_L)^T d, b = (dF/dW_R)^T d, each
  // without its A(W)^T d / 2 term. Those terms are linear in d and depend on
  // one side only, so a cell's two faces along an axis share one product
  // A(W)^T (d_west + d_east) (at_d) instead of taking one each.
  template <int D>
  __device__ __forceinline__ void face(const double* wl, const Prim& pl, const double* wr,
                                       const Prim& pr, const double* d, double* a,
                                       double* b) const {
    const double unl = D == 0 ? pl.u : pl.v;
    const double unr = D == 0 ? pr.u : pr.v;
    const double sl = fabs(unl) + pl.c;
    const double sr = fabs(unr) + pr.c;
    const bool left = sl >= sr;
    const double hs = 0.5 * (left ? sl : sr);
    // the faster side's primitives, selected field by field (a choice
    // between the two structs' addresses would put them in scratch memory)
    Prim q;
    q.r = left ? pl.r : pr.r;
    q.u = left ? pl.u : pr.u;
    q.v = left ? pl.v : pr.v;
    q.p = left ? pl.p : pr.p;
    q.c = left ? pl.c : pr.c;
    double gs[4];
    dspeed<D>(q, gs);
    const double dwd = fma(wr[0] - wl[0], d[0],
                           fma(wr[1] - wl[1], d[1],
                               fma(wr[2] - wl[2], d[2], (wr[3] - wl[3]) * d[3])));
    const double h = 0.5 * dwd;
    const double hl = left ? h : 0.0, hr = left ? 0.0 : h;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double t = hs * d[k];
      a[k] = fma(-hl, gs[k], t);
      b[k] = fma(-hr, gs[k], -t);
    }
  }
  __device__ __forceinline__ void shift_next(const double* w, const Prim& q, double* wr,
                                             Prim& qr) const {
#pragma unroll
    for (int v = 0; v < 4; ++v) wr[v] = from_next(w[v]);
    qr.r = from_next(q.r);
    qr.u = from_next(q.u);
    qr.v = from_next(q.v);
    qr.p = from_next(q.p);
    qr.c = from_next(q.c);
  }
};

template <int BC>
__device__ __forceinline__ int adj_col(int i, int nx) {
  int c;
  if (BC == 0) c = i < 0 ? i + nx : (i >= nx ? i - nx : i);
  else c = i;
  c = c < 0 ? 0 : c;
  return c >= nx ? nx - 1 : c;
}

template <int BC>
__device__ __forceinline__ int adj_row(int r, int ny) {
  if (BC == 0) return r < 0 ? ny - 1 : (r >= ny ? 0 : r);
  return r < 0 ? 0 : (r >= ny ? ny - 1 : r);
}

// State and multiplier of row r; the multiplier of a ghost row (or ghost
// column, `ghost_col`) is zero. With Dirichlet boundaries (BC 2) a ghost
// holds the prescribed state of its side (gh: ghost[side * kMaxVar + v];
// `col_side` is the side of a ghost column); with transmissive ones it is the
// boundary cell, loaded from the clamped index.
template <int NV, int BC>
__device__ __forceinline__ void load_adj_row(double* w, double* l, const double* __restrict__ wb,
                                             const double* __restrict__ lb, const GridGeom& g,
                                             int r, bool ghost_col, const double* gh = nullptr,
                                             int col_side = 0) {
  const size_t off = static_cast<size_t>(adj_row<BC>(r, g.ny)) * g.ld;
  const bool ghost_row = BC != 0 && (r < 0 || r >= g.ny);
  const bool ghost = ghost_col || ghost_row;
  const int side = ghost_row ? (r < 0 ? kSouth : kNorth) : col_side;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const double x = wb[v * g.plane + off];
    w[v] = (BC == kDirichlet && ghost) ? gh[side * kMaxVar + v] : x;
    const double y = lb[v * g.plane + off];
    l[v] = ghost ? 0.0 : y;
  }
}

// One strip of 62 cells, one per lane (lanes 0 and 63 only supply the halo
// cells): the layout for odd pitches and unaligned buffers. DOWN marches the
// rows from the top of the tile down instead of up: alternate tiles of a
// column run in opposite directions, so two vertically adjacent tiles reach
// the rows they share (one's last row, the other's halo row) at about the
// same time and the second read is served from L2. Every face is evaluated
// with the same arguments and every cell sums its shares in the same order
// in both directions, so the multipliers do not depend on it.
template <class M, int BC, bool DOWN = false>
__device__ __forceinline__ void adjoint_strip1(const M& m, const AdjointArgs& a, int xs, int j0,
                                               int j1, double mux, double muy) {
  constexpr int NV = M::NV;
  using Prim = typename M::Prim;
  const int lane = threadIdx.x & (kWave - 1);
  const GridGeom& g = a.g;
  const int i = xs - 1 + lane;
  const int ic = adj_col<BC>(i, g.nx);
  const bool out = (lane >= 1) & (lane <= kOutPerWave) & (i < g.nx);
  const bool ghost_col = BC != 0 && (i < 0 || i >= g.nx);
  const int col_side = i < 0 ? kWest : kEast;
  const double* gh = a.ghost;
  const bool west = BC == 1 && i == 0;
  const bool east = BC == 1 && i == g.nx - 1;
  const double kw = west ? 2.0 : 1.0, ke = east ? 2.0 : 1.0;
  const double* wb = a.w + ic;
  const double* lb = a.lam_in + ic;

  // Register ring of R = PF + 2 rows of (W, lambda): row j in slot c, the
  // next row in the march (j + S) in slot n, rows up to PF further loading
  // into the slot the row behind vacated. The row loop is unrolled R times
  // so every slot index is static; rows past the tile are computed from
  // loads clamped to its halo row and not stored.
  constexpr int PF = FVM_ADJ_PREFETCH;
  constexpr int R = PF + 2;
  constexpr int S = DOWN ? -1 : 1;
  const int jf = DOWN ? j1 - 1 : j0;   // the first row of the march
  const int jh = DOWN ? j0 - 1 : j1;   // the halo row past its last
  auto ahead = [&](int r) { return DOWN ? max(r, jh) : min(r, jh); };
  auto row = [&](double* w, double* l, int r) {
    load_adj_row<NV, BC>(w, l, wb, lb, g, r, ghost_col, gh, col_side);
  };
  // the face behind the current row (between it and the previous one in
  // the march): lower row's share Fl, upper row's share Fu, d = lam_upper -
  // lam_lower
  double W[R][NV], L[R][NV], Fl[NV], Fu[NV], Fd[NV];
  Prim P[R];
  row(W[R - 1], L[R - 1], jf - S);
  row(W[0], L[0], jf);
#pragma unroll
  for (int p = 1; p <= PF; ++p) row(W[p], L[p], ahead(jf + S * p));
  m.prim(W[R - 1], P[R - 1]);
  m.prim(W[0], P[0]);
  {
    const int lo = DOWN ? 0 : R - 1, up = DOWN ? R - 1 : 0;
#pragma unroll
    for (int v = 0; v < NV; ++v) Fd[v] = L[up][v] - L[lo][v];
    m.template face<1>(W[lo], P[lo], W[up], P[up], Fd, Fl, Fu);
  }

  for (int jb = jf; DOWN ? jb > jh : jb < jh; jb += S * R) {
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int j = jb + S * u;
      const int c = u, n = (u + 1) % R, l = (u + R - 1) % R;
      row(W[l], L[l], ahead(j + S * (1 + PF)));
      m.prim(W[n], P[n]);
      // the face ahead: north of row j going up, south of it going down
      double Gd[NV], Gl[NV], Gu[NV];
      const int glo = DOWN ? n : c, gup = DOWN ? c : n;
#pragma unroll
      for (int v = 0; v < NV; ++v) Gd[v] = L[gup][v] - L[glo][v];
      m.template face<1>(W[glo], P[glo], W[gup], P[gup], Gd, Gl, Gu);
      // row j's north face (its lower share An, the upper Bn, dn) and south
      // face (As, Bs, ds)
      const double* An = DOWN ? Fl : Gl;
      const double* Bn = DOWN ? Fu : Gu;
      const double* dn = DOWN ? Fd : Gd;
      const double* As = DOWN ? Gl : Fl;
      const double* Bs = DOWN ? Gu : Fu;
      const double* ds = DOWN ? Gd : Fd;
      double dx[NV], Wr[NV], Ax[NV], Bx[NV];
      Prim Pr;
      m.shift_next(W[c], P[c], Wr, Pr);
#pragma unroll
      for (int v = 0; v < NV; ++v) dx[v] = from_next(L[c][v]) - L[c][v];
      m.template face<0>(W[c], P[c], Wr, Pr, dx, Ax, Bx);
      const bool south = BC == 1 && j == 0;
      const bool north = BC == 1 && j == g.ny - 1;
      const size_t cell = static_cast<size_t>(j) * g.ld + ic;
      // A(W)^T of the sums of the cell's faces' d along each axis (a
      // transmissive ghost is a copy of the cell: its face counts twice)
      double gx[NV], gy[NV];
      if constexpr (M::kCellA) {
        double Dx[NV], Dy[NV];
        const double ks = south ? 2.0 : 1.0, kn = north ? 2.0 : 1.0;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const double dw = from_prev(dx[v]);  // the west face's d
          Dx[v] = fma(kw, dw, ke * dx[v]);
          Dy[v] = fma(ks, ds[v], kn * dn[v]);
        }
        m.template at_d<0>(W[c], P[c], Dx, gx);
        m.template at_d<1>(W[c], P[c], Dy, gy);
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const double bw = from_prev(Bx[v]);
        const double aw = from_prev(Ax[v]);
        double sx = Ax[v] + bw;
        if (west) sx += aw;
        if (east) sx += Bx[v];
        double sy = An[v] + Bs[v];
        if (south) sy += As[v];
        if (north) sy += Bn[v];
        if constexpr (M::kCellA) {
          sx = fma(0.5, gx[v], sx);
          sy = fma(0.5, gy[v], sy);
        }
        const double lo = L[c][v] + fma(mux, sx, muy * sy);
        if (out && j >= j0 && j < j1) a.lam_out[v * g.plane + cell] = lo;
      }
      // the face ahead is the next row's face behind; of its shares that
      // row needs only its own (its other face's ghost share applies at the
      // grid's first row alone)
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        Fl[v] = DOWN ? Gl[v] : 0.0;
        Fu[v] = DOWN ? 0.0 : Gu[v];
        Fd[v] = Gd[v];
      }
    }
  }
}

typedef double adj_dbl2 __attribute__((ext_vector_type(2)));

// One strip of 128 cells, two adjacent cells (a, b) per lane with 16-byte
// accesses. Faces: (a | b) inside the lane, (b | next lane's a) with the
// neighbour's state by DPP, and the strip's two end faces from a halo cell
// loaded by lanes 0 and 63. Every face is the one-cell strip's face with the
// same arguments, and each cell sums its shares in the same order, so the
// two layouts give bitwise the same multipliers. EDGE: the strip runs past
// column nx (cells there are clamped or wrapped, never stored; on a
// transmissive boundary they are ghost cells with a zero multiplier).
template <class M, int BC, bool EDGE>
__device__ __forceinline__ void adjoint_strip2(const M& m, const AdjointArgs& a, int xs, int j0,
                                               int j1, double mux, double muy) {
  constexpr int NV = M::NV;
  using Prim = typename M::Prim;
  const GridGeom& g = a.g;
  const int lane = threadIdx.x & (kWave - 1);
  const bool first = lane == 0, last = lane == kWave - 1;
  const int xa = xs + 2 * lane, xb = xa + 1;
  const int ca = EDGE ? adj_col<BC>(xa, g.nx) : xa;
  const int cb = EDGE ? adj_col<BC>(xb, g.nx) : xb;
  const bool oka = !EDGE || xa < g.nx, okb = !EDGE || xb < g.nx;
  const bool gca = BC != 0 && EDGE && xa >= g.nx;
  const bool gcb = BC != 0 && EDGE && xb >= g.nx;
  const int hx = first ? xs - 1 : xs + 2 * kWave;  // halo column of lanes 0 and 63
  const int ch = adj_col<BC>(hx, g.nx);
  const bool gch = BC != 0 && (hx < 0 || hx >= g.nx);
  const int h_side = hx < 0 ? kWest : kEast;
  const double* gh = a.ghost;
  const bool west = BC == 1 && xa == 0;
  const bool east_a = BC == 1 && xa == g.nx - 1;
  const bool east_b = BC == 1 && xb == g.nx - 1;
  const double kwa = west ? 2.0 : 1.0, kea = east_a ? 2.0 : 1.0, keb = east_b ? 2.0 : 1.0;

  auto prow = [&](double* wa, double* wbv, double* la, double* lbv, int r) {
    const size_t off = static_cast<size_t>(adj_row<BC>(r, g.ny)) * g.ld;
    const bool grow = BC != 0 && (r < 0 || r >= g.ny);
    const int rs = r < 0 ? kSouth : kNorth;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const size_t base = v * g.plane + off;
      if (!EDGE) {
        const adj_dbl2 w2 = *reinterpret_cast<const adj_dbl2*>(a.w + base + ca);
        const adj_dbl2 l2 = *reinterpret_cast<const adj_dbl2*>(a.lam_in + base + ca);
        wa[v] = w2.x;
        wbv[v] = w2.y;
        la[v] = grow ? 0.0 : l2.x;
        lbv[v] = grow ? 0.0 : l2.y;
      } else {
        wa[v] = a.w[base + ca];
        wbv[v] = a.w[base + cb];
        const double x = a.lam_in[base + ca], y = a.lam_in[base + cb];
        la[v] = (grow || gca) ? 0.0 : x;
        lbv[v] = (grow || gcb) ? 0.0 : y;
      }
      if constexpr (BC == kDirichlet) {
        // ghost rows, then ghost columns past the east edge (corners are
        // never used)
        if (grow) {
          wa[v] = gh[rs * kMaxVar + v];
          wbv[v] = gh[rs * kMaxVar + v];
        } else {
          if (gca) wa[v] = gh[kEast * kMaxVar + v];
          if (gcb) wbv[v] = gh[kEast * kMaxVar + v];
        }
      }
    }
  };
  auto hrow = [&](double* wh, double* lh, int r) {
    const size_t off = static_cast<size_t>(adj_row<BC>(r, g.ny)) * g.ld + ch;
    const bool grow = BC != 0 && (r < 0 || r >= g.ny);
    const bool ghost = gch || grow;
    const int side = grow ? (r < 0 ? kSouth : kNorth) : h_side;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const double x = a.w[v * g.plane + off];
      wh[v] = (BC == kDirichlet && ghost) ? gh[side * kMaxVar + v] : x;
      const double y = a.lam_in[v * g.plane + off];
      lh[v] = ghost ? 0.0 : y;
    }
  };

  constexpr int PF = FVM_ADJ_PREFETCH2;
  constexpr int R = PF + 2;
  double WA[R][NV], WB[R][NV], LA[R][NV], LB[R][NV], WH[R][NV], LH[R][NV];
  double BsA[NV], BsB[NV], AsA[NV], AsB[NV], DsA[NV], DsB[NV];
  Prim PA[R], PB[R];
  prow(WA[R - 1], WB[R - 1], LA[R - 1], LB[R - 1], j0 - 1);
  prow(WA[0], WB[0], LA[0], LB[0], j0);
  hrow(WH[0], LH[0], j0);
#pragma unroll
  for (int p = 1; p <= PF; ++p) {
    prow(WA[p], WB[p], LA[p], LB[p], min(j0 + p, j1));
    hrow(WH[p], LH[p], min(j0 + p, j1 - 1));
  }
  m.prim(WA[R - 1], PA[R - 1]);
  m.prim(WB[R - 1], PB[R - 1]);
  m.prim(WA[0], PA[0]);
  m.prim(WB[0], PB[0]);
  {
    double d[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) d[v] = DsA[v] = LA[0][v] - LA[R - 1][v];
    m.template face<1>(WA[R - 1], PA[R - 1], WA[0], PA[0], d, AsA, BsA);
#pragma unroll
    for (int v = 0; v < NV; ++v) d[v] = DsB[v] = LB[0][v] - LB[R - 1][v];
    m.template face<1>(WB[R - 1], PB[R - 1], WB[0], PB[0], d, AsB, BsB);
  }

  for (int jb = j0; jb < j1; jb += R) {
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int j = jb + u;
      const int c = u, n = (u + 1) % R, l = (u + R - 1) % R;
      prow(WA[l], WB[l], LA[l], LB[l], min(j + 1 + PF, j1));
      hrow(WH[l], LH[l], min(j + 1 + PF, j1 - 1));
      m.prim(WA[n], PA[n]);
      m.prim(WB[n], PB[n]);
      double dyA[NV], dyB[NV], AyA[NV], ByA[NV], AyB[NV], ByB[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) dyA[v] = LA[n][v] - LA[c][v];
      m.template face<1>(WA[c], PA[c], WA[n], PA[n], dyA, AyA, ByA);
#pragma unroll
      for (int v = 0; v < NV; ++v) dyB[v] = LB[n][v] - LB[c][v];
      m.template face<1>(WB[c], PB[c], WB[n], PB[n], dyB, AyB, ByB);
      // (a | b)
      double dab[NV], Aab[NV], Bab[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) dab[v] = LB[c][v] - LA[c][v];
      m.template face<0>(WA[c], PA[c], WB[c], PB[c], dab, Aab, Bab);
      // (b | next lane's a); lane 63's is replaced by its halo face below
      double dr[NV], Wr[NV], Ar[NV], Br[NV];
      Prim Pr;
      m.shift_next(WA[c], PA[c], Wr, Pr);
#pragma unroll
      for (int v = 0; v < NV; ++v) dr[v] = from_next(LA[c][v]) - LB[c][v];
      m.template face<0>(WB[c], PB[c], Wr, Pr, dr, Ar, Br);
      // the strip's end faces: lane 0 (halo | a), lane 63 (b | halo)
      double dh[NV], Wl[NV], Wt[NV], Ah[NV], Bh[NV];
      Prim Ph;
      m.prim(WH[c], Ph);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        Wl[v] = first ? WH[c][v] : WB[c][v];
        Wt[v] = first ? WA[c][v] : WH[c][v];
        dh[v] = (first ? LA[c][v] : LH[c][v]) - (first ? LH[c][v] : LB[c][v]);
      }
      const Prim Pl = first ? Ph : PB[c];
      const Prim Pt = first ? PA[c] : Ph;
      m.template face<0>(Wl, Pl, Wt, Pt, dh, Ah, Bh);
      const bool south = BC == 1 && j == 0;
      const bool north = BC == 1 && j == g.ny - 1;
      // A(W)^T of the sums of each cell's faces' d, formed as in the
      // one-cell strip (a transmissive ghost's face counts twice)
      double gxa[NV], gxb[NV], gya[NV], gyb[NV];
      if constexpr (M::kCellA) {
        double Dxa[NV], Dxb[NV], Dya[NV], Dyb[NV];
        const double ks = south ? 2.0 : 1.0, kn = north ? 2.0 : 1.0;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const double dp = from_prev(dr[v]);
          const double dwa = first ? dh[v] : dp;  // a's west face
          const double deb = last ? dh[v] : dr[v];  // b's east face
          Dxa[v] = fma(kwa, dwa, kea * dab[v]);
          Dxb[v] = fma(1.0, dab[v], keb * deb);
          Dya[v] = fma(ks, DsA[v], kn * dyA[v]);
          Dyb[v] = fma(ks, DsB[v], kn * dyB[v]);
        }
        m.template at_d<0>(WA[c], PA[c], Dxa, gxa);
        m.template at_d<0>(WB[c], PB[c], Dxb, gxb);
        m.template at_d<1>(WA[c], PA[c], Dya, gya);
        m.template at_d<1>(WB[c], PB[c], Dyb, gyb);
      }
      double OA[NV], OB[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        // the cross-lane moves run with every lane active
        const double bp = from_prev(Br[v]);
        const double ap = from_prev(Ar[v]);
        const double lB = first ? Bh[v] : bp;  // a's west face: a's share
        const double lA = first ? Ah[v] : ap;  // ... and the west cell's
        const double rA = last ? Ah[v] : Ar[v];  // b's east face: b's share
        const double rB = last ? Bh[v] : Br[v];  // ... and the east cell's
        double sxa = Aab[v] + lB;
        if (west) sxa += lA;
        if (east_a) sxa += Bab[v];
        double sxb = rA + Bab[v];
        if (east_b) sxb += rB;
        double sya = AyA[v] + BsA[v];
        if (south) sya += AsA[v];
        if (north) sya += ByA[v];
        double syb = AyB[v] + BsB[v];
        if (south) syb += AsB[v];
        if (north) syb += ByB[v];
        if constexpr (M::kCellA) {
          sxa = fma(0.5, gxa[v], sxa);
          sxb = fma(0.5, gxb[v], sxb);
          sya = fma(0.5, gya[v], sya);
          syb = fma(0.5, gyb[v], syb);
        }
        OA[v] = LA[c][v] + fma(mux, sxa, muy * sya);
        OB[v] = LB[c][v] + fma(mux, sxb, muy * syb);
      }
      if (j < j1) {
        const size_t row = static_cast<size_t>(j) * g.ld;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          double* o = a.lam_out + v * g.plane + row;
          if (!EDGE) {
            const adj_dbl2 x = {OA[v], OB[v]};
            *reinterpret_cast<adj_dbl2*>(o + ca) = x;
          } else {
            if (oka) o[ca] = OA[v];
            if (okb) o[cb] = OB[v];
          }
        }
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        BsA[v] = ByA[v];
        BsB[v] = ByB[v];
        AsA[v] = 0.0;
        AsB[v] = 0.0;
        DsA[v] = dyA[v];
        DsB[v] = dyB[v];
      }
    }
  }
}

}  // namespace fvm
