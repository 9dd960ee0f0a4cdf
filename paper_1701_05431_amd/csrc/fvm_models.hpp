// fvm_models.hpp -- pointwise physics of the three models (and the spray's
// transport-only variant), device side.
//
// Each model provides
//   Prim              per-cell derived quantities reused by both face fluxes;
//   prim(w, P)        W -> Prim;
//   flux<D>(wl,pl,wr,pr,f)  numerical flux across a face with axis normal D
//                     (0 = x, 1 = y); left = lower index;
//   shift_next(w,p,wr,pr)   the right neighbour's (W, Prim) from lane+1;
//   pick(t, a, b)     t ? a : b for two Prims, field by field;
//   speeds(w, sx, sy) largest |eigenvalue| along x and y of a new state, NaN
//                     when the state is non-finite or non-physical;
//   source(w, ugx, ugy, dt) the split source step (spray only);
//   kSource           whether the step kernel applies source() (the spray
//                     with the lognormal closure) or not;
//   kCommit           whether the step kernel reduces the new state's speeds
//                     and sets the next dt (all but the spray's transport-only
//                     step, whose source pass does it).
#pragma once

#include <hip/hip_runtime.h>

#include "fvm_internal.hpp"

// Rows of loads kept in flight per wave strip (register ring depth), for
// the two-cells-per-lane layout
#ifndef FVM_PREFETCH2_ADV
#define FVM_PREFETCH2_ADV 2
#endif
#ifndef FVM_PREFETCH2_EULER
#define FVM_PREFETCH2_EULER 2
#endif
#ifndef FVM_PREFETCH2_SPRAY
#define FVM_PREFETCH2_SPRAY 0  // no ring of loads in flight: two waves per SIMD instead
#endif
// ... and for the aligned one-cell-per-lane layout
#ifndef FVM_PREFETCH1_ADV
#define FVM_PREFETCH1_ADV 2
#endif
#ifndef FVM_PREFETCH1_EULER
#define FVM_PREFETCH1_EULER 1
#endif
#ifndef FVM_PREFETCH1_SPRAY
#define FVM_PREFETCH1_SPRAY 1
#endif

namespace fvm {

// ---- cross-lane moves ------------------------------------------------------
// Lane l receives lane l+1's value (wave_shl:1 DPP), resp. lane l-1's value
// (wave_shr:1). The edge lanes receive 0; the kernels never use those lanes'
// results.
__device__ __forceinline__ int dpp_from_next_i32(int x) {
  return __builtin_amdgcn_update_dpp(0, x, 0x130, 0xF, 0xF, false);
}
__device__ __forceinline__ int dpp_from_prev_i32(int x) {
  return __builtin_amdgcn_update_dpp(0, x, 0x138, 0xF, 0xF, false);
}
__device__ __forceinline__ double from_next(double x) {
#if FVM_SHUFFLE_WITH_BPERMUTE
  return __shfl_down(x, 1, 64);
#else
  const long long b = __double_as_longlong(x);
  const int lo = dpp_from_next_i32(static_cast<int>(b));
  const int hi = dpp_from_next_i32(static_cast<int>(b >> 32));
  return __longlong_as_double((static_cast<long long>(hi) << 32) |
                              static_cast<unsigned int>(lo));
#endif
}
__device__ __forceinline__ double from_prev(double x) {
#if FVM_SHUFFLE_WITH_BPERMUTE
  return __shfl_up(x, 1, 64);
#else
  const long long b = __double_as_longlong(x);
  const int lo = dpp_from_prev_i32(static_cast<int>(b));
  const int hi = dpp_from_prev_i32(static_cast<int>(b >> 32));
  return __longlong_as_double((static_cast<long long>(hi) << 32) |
                              static_cast<unsigned int>(lo));
#endif
}

__device__ __forceinline__ bool finite(double x) { return __builtin_isfinite(x); }

// Reciprocal and square root of the per-cell primitives. With
// FVM_FAST_DIVSQRT (the default) the hardware estimates are refined in FP64:
// two Newton-Raphson steps for 1/x, and for sqrt(x) one step of Goldschmidt's
// coupled iteration on (x*y, y/2), y ~ 1/sqrt(x), followed by one
// Newton-style residual correction (the textbook scheme, e.g. P. Markstein,
// IA-64 and Elementary Functions, 2000). For the normal-range arguments the
// models produce this is within an ulp of the correctly rounded result, in
// about half the instructions. Zero, negative and non-finite arguments are
// classified as by the exact forms (0 -> 0 for the root, NaN propagates).
// FVM_FAST_DIVSQRT=0 selects the compiler's correctly rounded sequences.
#ifndef FVM_FAST_DIVSQRT
#define FVM_FAST_DIVSQRT 1
#endif
__device__ __forceinline__ double recip(double x) {
#if FVM_FAST_DIVSQRT
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
#else
  return 1.0 / x;
#endif
}
__device__ __forceinline__ double root(double x) {
#if FVM_FAST_DIVSQRT
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y;
  double h = 0.5 * y;
  const double r = fma(-h, g, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  const double d = fma(-g, g, x);
  g = fma(d, h, g);
  return x == 0.0 ? x : g;
#else
  return sqrt(x);
#endif
}

// 1/sqrt(x) for a positive normal argument: the hardware estimate refined by
// two Newton-Raphson steps y <- y + y (1 - x y^2) / 2 (each squares the
// relative error), or the exact quotient with FVM_FAST_DIVSQRT=0.
__device__ __forceinline__ double rroot(double x) {
#if FVM_FAST_DIVSQRT
  double y = __builtin_amdgcn_rsq(x);
  double e = fma(-x * y, y, 1.0);
  y = fma(0.5 * y, e, y);
  e = fma(-x * y, y, 1.0);
  return fma(0.5 * y, e, y);
#else
  return 1.0 / sqrt(x);
#endif
}

// Natural logarithm of a positive finite argument (the spray closure's
// moment ratios), from the series log(m) = 2 atanh(s) = 2 (s + s^3/3 + s^5/5
// + ...), s = (m - 1) / (m + 1), after splitting x = m 2^e with m in
// [sqrt(1/2), sqrt(2)): there |s| <= 0.1716, and the terms through s^19
// leave a truncation error below 3e-17 relative. e ln 2 is added in two
// parts (ln 2 rounded to 32 significant bits, so e times it is exact, and
// the remainder). Within about two ulps of the correctly rounded logarithm
// in some 30 instructions; with FVM_FAST_LOG=0, the library's log.
#ifndef FVM_FAST_LOG
#define FVM_FAST_LOG 1
#endif
__device__ __forceinline__ double logd(double x) {
#if FVM_FAST_LOG
  constexpr double kLn2Hi = 0.6931471806019545;     // ln 2 to 32 significant bits
  constexpr double kLn2Lo = -4.2009150726810846e-11;  // ln 2 - kLn2Hi
  int e;
  double m = frexp(x, &e);  // x = m 2^e, m in [1/2, 1)
  const bool small = m < 0.7071067811865476;
  m = small ? 2.0 * m : m;
  e = small ? e - 1 : e;
  const double f = m - 1.0;  // exact: m lies within a factor 2 of 1
  const double s = f * recip(2.0 + f);
  const double z = s * s;
  double p = 2.0 / 19.0;
  p = fma(p, z, 2.0 / 17.0);
  p = fma(p, z, 2.0 / 15.0);
  p = fma(p, z, 2.0 / 13.0);
  p = fma(p, z, 2.0 / 11.0);
  p = fma(p, z, 2.0 / 9.0);
  p = fma(p, z, 2.0 / 7.0);
  p = fma(p, z, 2.0 / 5.0);
  p = fma(p, z, 2.0 / 3.0);
  const double r = fma(s * z, p, 2.0 * s);  // 2 atanh(s)
  const double ed = static_cast<double>(e);
  return fma(ed, kLn2Hi, fma(ed, kLn2Lo, r));
#else
  return log(x);
#endif
}

// Index of the wave inside its workgroup, as a scalar: branches on it are
// uniform, so the strip code (and its DPP moves) runs with the whole wave
// active.
__device__ __forceinline__ int wave_index() {
  return __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) / kWave);
}

// ---- linear advection --------------------------------------------------------
// u_t + a.grad u = 0; upwind flux a+ u_L + a- u_R (the Lax-Friedrichs flux of
// a linear flux in exact arithmetic).
struct Adv {
  static constexpr int NV = 1;
  static constexpr bool kSource = false;  // no pointwise source
  static constexpr bool kCommit = true;   // the step reduces speeds and sets the next dt
  static constexpr int kPrefetch2 = FVM_PREFETCH2_ADV;
  static constexpr int kPrefetch1 = FVM_PREFETCH1_ADV;
  struct Prim {};
  __device__ static Prim pick(bool, const Prim&, const Prim&) { return {}; }
  double ax, ay;
  __device__ explicit Adv(const ModelConsts& m) : ax(m.ax), ay(m.ay) {}
  __device__ __forceinline__ void prim(const double*, Prim&) const {}
  template <int D>
  __device__ __forceinline__ void flux(const double* wl, const Prim&, const double* wr,
                                       const Prim&, double* f) const {
    const double a = D == 0 ? ax : ay;
    const double ap = a > 0.0 ? a : 0.0;
    const double am = a < 0.0 ? a : 0.0;
    f[0] = fma(ap, wl[0], am * wr[0]);
  }
  __device__ __forceinline__ void shift_next(const double* w, const Prim&, double* wr,
                                             Prim&) const {
    wr[0] = from_next(w[0]);
  }
  __device__ __forceinline__ void speeds(const double* w, double& sx, double& sy) const {
    const bool ok = finite(w[0]);
    sx = ok ? fabs(ax) : __builtin_nan("");
    sy = ok ? fabs(ay) : __builtin_nan("");
  }
};

// ---- Euler equations of a perfect gas (Sec. 5) -------------------------------
// W = (rho, rho u, rho v, rho E), p = (gamma-1)(rho E - rho (u^2+v^2)/2),
// c^2 = gamma p / rho, eigenvalues u.n - c, u.n, u.n, u.n + c; Rusanov flux
// F~ = (F(W_L).n + F(W_R).n)/2 - sigma/2 (W_R - W_L),
// sigma = max(|u_L.n| + c_L, |u_R.n| + c_R)  (Sec. 2.2.1).
struct Euler {
  static constexpr int NV = 4;
  static constexpr bool kSource = false;
  static constexpr bool kCommit = true;
  static constexpr int kPrefetch2 = FVM_PREFETCH2_EULER;
  static constexpr int kPrefetch1 = FVM_PREFETCH1_EULER;
  struct Prim { double u, v, p, c; };
  // t ? a : b, field by field (registers, not a choice of address)
  __device__ static Prim pick(bool t, const Prim& a, const Prim& b) {
    return {t ? a.u : b.u, t ? a.v : b.v, t ? a.p : b.p, t ? a.c : b.c};
  }
  double gamma, gm1;
  __device__ explicit Euler(const ModelConsts& m) : gamma(m.gamma), gm1(m.gm1) {}
  __device__ __forceinline__ void prim(const double* w, Prim& q) const {
    const double r = recip(w[0]);
    q.u = w[1] * r;
    q.v = w[2] * r;
    q.p = gm1 * fma(-0.5, fma(w[1], q.u, w[2] * q.v), w[3]);
    q.c = root(gamma * q.p * r);
  }
  template <int D>
  __device__ __forceinline__ void flux(const double* wl, const Prim& pl, const double* wr,
                                       const Prim& pr, double* f) const {
    const double unl = D == 0 ? pl.u : pl.v;
    const double unr = D == 0 ? pr.u : pr.v;
    const double sl = fabs(unl) + pl.c;
    const double sr = fabs(unr) + pr.c;
    const double sig = sl >= sr ? sl : sr;
    const double hs = 0.5 * sig;
    // physical fluxes: (rho u_n, rho u u_n + p n_x, rho v u_n + p n_y, (rho E + p) u_n)
    const double l0 = wl[1 + D], r0 = wr[1 + D];
    const double l1 = D == 0 ? fma(wl[1], unl, pl.p) : wl[1] * unl;
    const double r1 = D == 0 ? fma(wr[1], unr, pr.p) : wr[1] * unr;
    const double l2 = D == 1 ? fma(wl[2], unl, pl.p) : wl[2] * unl;
    const double r2 = D == 1 ? fma(wr[2], unr, pr.p) : wr[2] * unr;
    const double l3 = (wl[3] + pl.p) * unl, r3 = (wr[3] + pr.p) * unr;
    f[0] = fma(-hs, wr[0] - wl[0], 0.5 * (l0 + r0));
    f[1] = fma(-hs, wr[1] - wl[1], 0.5 * (l1 + r1));
    f[2] = fma(-hs, wr[2] - wl[2], 0.5 * (l2 + r2));
    f[3] = fma(-hs, wr[3] - wl[3], 0.5 * (l3 + r3));
  }
  __device__ __forceinline__ void shift_next(const double* w, const Prim& q, double* wr,
                                             Prim& qr) const {
#pragma unroll
    for (int v = 0; v < 4; ++v) wr[v] = from_next(w[v]);
    qr.u = from_next(q.u);
    qr.p = from_next(q.p);
    qr.c = from_next(q.c);
    qr.v = 0.0;  // the x-flux does not use v
  }
  __device__ __forceinline__ void speeds(const double* w, double& sx, double& sy) const {
    Prim q;
    prim(w, q);
    const bool ok = finite(w[0]) && finite(w[1]) && finite(w[2]) && finite(w[3]) &&
                    (w[0] > 0.0) && (q.p >= 0.0);
    sx = ok ? fabs(q.u) + q.c : __builtin_nan("");
    sy = ok ? fabs(q.v) + q.c : __builtin_nan("");
  }
};

// ---- evaporating spray, six fractional moments (Sec. 6.1) --------------------
// W = (m_0, m_{1/2}, m_{2/2}, m_{3/2}, q_x, q_y), u = q / m_{2/2}; kinetic
// upwind flux W_L (u_L.n)+ + W_R (u_R.n)-; source: evaporation of the moments
// (-K n(0), -K/2 m_{-1/2}, -K m_0, -3K/2 m_{1/2}, -K m_0 u) and drag
// m_0 (u_g - u)/theta, with n(0) and m_{-1/2} from a lognormal fit to
// (m_0, m_{1/2}, m_{2/2}).
struct Spray {
  static constexpr int NV = 6;
  static constexpr bool kSource = true;   // the lognormal-closure source, fused
  static constexpr bool kCommit = true;
  static constexpr int kPrefetch2 = FVM_PREFETCH2_SPRAY;
  static constexpr int kPrefetch1 = FVM_PREFETCH1_SPRAY;
  struct Prim { double ux, uy; };
  __device__ static Prim pick(bool t, const Prim& a, const Prim& b) {
    return {t ? a.ux : b.ux, t ? a.uy : b.uy};
  }
  double K, inv_theta, s_eps, log_s_eps;
  __device__ explicit Spray(const ModelConsts& m)
      : K(m.K), inv_theta(m.inv_theta), s_eps(m.s_eps), log_s_eps(m.log_s_eps) {}
  __device__ __forceinline__ void prim(const double* w, Prim& q) const {
    const bool ok = w[2] > 1e-300;
    const double r = recip(ok ? w[2] : 1.0);
    q.ux = ok ? w[4] * r : 0.0;
    q.uy = ok ? w[5] * r : 0.0;
  }
  template <int D>
  __device__ __forceinline__ void flux(const double* wl, const Prim& pl, const double* wr,
                                       const Prim& pr, double* f) const {
    const double ul = D == 0 ? pl.ux : pl.uy;
    const double ur = D == 0 ? pr.ux : pr.uy;
    const double up = ul > 0.0 ? ul : 0.0;
    const double um = ur < 0.0 ? ur : 0.0;
#pragma unroll
    for (int k = 0; k < 6; ++k) f[k] = fma(wl[k], up, wr[k] * um);
  }
  __device__ __forceinline__ void shift_next(const double* w, const Prim& q, double* wr,
                                             Prim& qr) const {
#pragma unroll
    for (int v = 0; v < 6; ++v) wr[v] = from_next(w[v]);
    qr.ux = from_next(q.ux);
    qr.uy = 0.0;
  }
  __device__ __forceinline__ void speeds(const double* w, double& sx, double& sy) const {
    Prim q;
    prim(w, q);
    bool ok = finite(w[4]) && finite(w[5]);
#pragma unroll
    for (int k = 0; k < 4; ++k) ok = ok & finite(w[k]) & (w[k] >= 0.0);
    sx = ok ? fabs(q.ux) : __builtin_nan("");
    sy = ok ? fabs(q.uy) : __builtin_nan("");
  }
  // W <- W + dt S(W)
  __device__ __forceinline__ void source(double* w, double ugx, double ugy, double dt) const {
    const double m0 = w[0], m1 = w[1], m2 = w[2];
    if (!(m0 > 1e-300) || !(m1 > 1e-300) || !(m2 > 1e-300)) return;
    const double r2 = recip(m2);
    const double ux = w[4] * r2, uy = w[5] * r2;
    const double r0 = recip(m0);
    const double L1 = logd(m1 * r0);
    const double L2 = logd(m2 * r0);
    double s2 = 4.0 * fma(-2.0, L1, L2);
    s2 = s2 < 1e-8 ? 1e-8 : s2;
    const double mu = fma(2.0, L1, -0.25 * s2);
    const double mmh = m0 * exp(fma(-0.5, mu, 0.125 * s2));
    // n(S_eps) = m_0 exp(-z^2 / (2 s^2)) / (S_eps sqrt(2 pi s^2)), z = ln S_eps - mu,
    // with 1/S_eps folded into the exponential
    const double z = log_s_eps - mu;
    const double rs = rroot(6.283185307179586 * s2);
    const double is2 = 6.283185307179586 * (rs * rs);
    const double n0 = m0 * rs * exp(fma(-(z * z), 0.5 * is2, -log_s_eps));
    const double Km0 = K * m0;
    w[0] = fma(dt, -K * n0, m0);
    w[1] = fma(dt, -(0.5 * K) * mmh, m1);
    w[2] = fma(dt, -Km0, m2);
    w[3] = fma(dt, -(1.5 * K) * m1, w[3]);
    w[4] = fma(dt, fma(-Km0, ux, m0 * (ugx - ux) * inv_theta), w[4]);
    w[5] = fma(dt, fma(-Km0, uy, m0 * (ugy - uy) * inv_theta), w[5]);
  }
};

// The spray transport alone: the step kernel writes W* and neither applies
// the source nor reduces the speeds; the entropy-maximising source pass
// (fvm_maxent.hip) then completes the step, reduces the speeds of W^{n+1}
// and sets the next dt.
struct SprayTransport : Spray {
  static constexpr int kPrefetch2 = 1;
  static constexpr bool kSource = false;
  static constexpr bool kCommit = false;
  __device__ explicit SprayTransport(const ModelConsts& m) : Spray(m) {}
};

}  // namespace fvm
