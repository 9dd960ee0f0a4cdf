// fvm_maxent.hip -- the spray source with the entropy-maximising closure
// (Sec. 6.1 eq. Essadki, Sec. 6.2).
//
// The evaporation terms need n(S=0) and m_{-1/2}, which the moments
// m_{0/2..3/2} do not determine; the paper takes them from the size
// distribution of largest entropy with those moments (the algorithm is in a
// reference it cites). With x = S^{1/2} that distribution is
// n(S) = exp(l0 + l1 x + l2 x^2 + l3 x^3) on S in [0, 1]; its multipliers
// minimise the convex dual Phi(l) = int n dS - sum_k l_k m_{k/2}, whose
// gradient is the moment mismatch and whose Hessian is the 4 x 4 matrix of
// the moments m_{(k+l)/2}. Each cell runs Newton's method on Phi from the
// normal density in x with the cell's mean and variance of x, or from the
// cell's multipliers of the previous pass when the caller keeps them (steps
// cut back until Phi decreases while the mismatch is large), with every moment
// integral taken by a composite 8-point Gauss-Legendre rule over 16 panels of
// x. Then n(S=0) = exp(l0) and m_{-1/2} = int S^{-1/2} n dS.
//
// The pass runs after the transport-only step kernel: per cell it reads W*
// and the gas velocity, writes W^{n+1} = W* + dt S(W*) in place, and reduces
// the speeds of W^{n+1} into the grid's maxima; its last workgroup sets the
// next dt (the step kernel's epilogue, moved here). Work per cell is some
// tens of thousands of FP64 operations against 112 bytes of traffic: the pass
// is bound by the FP64 vector units, not by HBM. A cell whose moments the
// closure cannot match becomes NaN, which the speed reduction reports.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstdint>

#include "fvm_adjoint_spray.hpp"
#include "fvm_host.hpp"
#include "fvm_internal.hpp"
#include "fvm_models.hpp"
#include "fvm_step.hpp"

namespace fvm {

// Quadrature nodes evaluated per unrolled loop step, and the minimum number
// of waves per SIMD the source pass is compiled for (0: the compiler's
// choice).
#ifndef FVM_MAXENT_UNROLL
#define FVM_MAXENT_UNROLL 8
#endif
#ifndef FVM_MAXENT_WAVES
#define FVM_MAXENT_WAVES 0
#endif

constexpr int kMePanels = 16;
constexpr int kMeThreads = 256;
constexpr int kMeMaxBlocks = 8192;

// m[j] = int S^{(j-1)/2} n dS = 2 int x^j e^{p(x)} dx for j = 0..7: m[0] is
// m_{-1/2}, m[1..4] the model's moments, m[5..7] the higher ones the Hessian
// needs.
__device__ __forceinline__ void me_moments(const double* l, const MaxEntRule& r, double* m) {
#pragma unroll
  for (int j = 0; j < 8; ++j) m[j] = 0.0;
  constexpr double h = 1.0 / kMePanels;
  for (int p = 0; p < kMePanels; ++p) {
#pragma unroll FVM_MAXENT_UNROLL
    for (int q = 0; q < 8; ++q) {
      const double x = fma(r.x[q], h, p * h);
      const double poly = fma(fma(fma(l[3], x, l[2]), x, l[1]), x, l[0]);
      const double e = (2.0 * h) * r.w[q] * exp(poly);
      double xp = e;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        m[j] += xp;
        xp *= x;
      }
    }
  }
}

// Newton direction: solves H d = -g with H_kl = mu[k+l+1] by Cholesky;
// false if H is not positive definite.
__device__ __forceinline__ bool me_direction(const double* mu, const double* g, double* d) {
  double L[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      double s = mu[i + j + 1];
#pragma unroll
      for (int k = 0; k < j; ++k) s = fma(-L[i][k], L[j][k], s);
      if (i == j) {
        if (!(s > 0.0)) return false;
        L[i][i] = sqrt(s);
      } else {
        L[i][j] = s / L[j][j];
      }
    }
  double y[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    double s = -g[i];
#pragma unroll
    for (int k = 0; k < i; ++k) s = fma(-L[i][k], y[k], s);
    y[i] = s / L[i][i];
  }
#pragma unroll
  for (int i = 3; i >= 0; --i) {
    double s = y[i];
#pragma unroll
    for (int k = i + 1; k < 4; ++k) s = fma(-L[k][i], d[k], s);
    d[i] = s / L[i][i];
  }
  return true;
}

// Newton's method on the dual from the multipliers l (in/out): true with
// (m_{-1/2}, n(S=0)) once the relative moment mismatch is <= 1e-14, or
// <= 1e-12 when a step no longer halves it; false if the moments cannot be
// matched from this start.
__device__ bool maxent_newton(const double* w, const MaxEntRule& r, double* l, double& mmh,
                              double& n0) {
  double mu[8];
  me_moments(l, r, mu);
  double prev = INFINITY;
  for (int it = 0; it < 100; ++it) {
    double g[4], rel = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      g[k] = mu[k + 1] - w[k];
      const double q = fabs(g[k]) / w[k];
      rel = q <= rel ? rel : q;  // NaN-sticky
    }
    if (!(rel == rel)) return false;
    if (rel <= 1e-14 || (rel <= 1e-12 && rel > 0.5 * prev)) {
      mmh = mu[0];
      n0 = exp(l[0]);
      return true;
    }
    prev = rel;
    double d[4];
    if (!me_direction(mu, g, d)) return false;
    double t = 1.0, trial[4], mt[8];
    if (rel > 1e-3) {
      // backtracking until Phi decreases by at least 1e-4 t g.d
      double phi = mu[1], slope = 0.0;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        phi = fma(-l[k], w[k], phi);
        slope = fma(g[k], d[k], slope);
      }
      bool accepted = false;
      for (int ls = 0; ls < 60 && !accepted; ++ls) {
#pragma unroll
        for (int k = 0; k < 4; ++k) trial[k] = fma(t, d[k], l[k]);
        me_moments(trial, r, mt);
        double pt = mt[1];
#pragma unroll
        for (int k = 0; k < 4; ++k) pt = fma(-trial[k], w[k], pt);
        if (pt <= phi + 1e-4 * t * slope)
          accepted = true;
        else
          t *= 0.5;
      }
      if (!accepted) return false;
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k) trial[k] = l[k] + d[k];
      me_moments(trial, r, mt);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) l[k] = trial[k];
#pragma unroll
    for (int j = 0; j < 8; ++j) mu[j] = mt[j];
  }
  return false;
}

// (m_{-1/2}, n(S=0)) of the entropy maximiser with moments w[0..3]. With
// `warm`, Newton starts from the multipliers in l (the cell's previous
// ones); otherwise, or if that fails, from the normal density in x with the
// cell's mean and variance of x. l returns the converged multipliers. False
// if the moments cannot be matched.
__device__ bool maxent_closure(const double* w, const MaxEntRule& r, bool warm, double* l,
                               double& mmh, double& n0) {
  if (warm && finite(l[0]) && finite(l[1]) && finite(l[2]) && finite(l[3])) {
    double t[4] = {l[0], l[1], l[2], l[3]};
    if (maxent_newton(w, r, t, mmh, n0)) {
#pragma unroll
      for (int k = 0; k < 4; ++k) l[k] = t[k];
      return true;
    }
  }
  const double a = w[1] / w[0];
  const double var = w[2] / w[0] - a * a;
  if (!(var > 0.0)) return false;
  double c[4] = {0.0, a / var, -0.5 / var, 0.0}, mu[8];
  me_moments(c, r, mu);
  if (!(mu[1] > 0.0)) return false;
  c[0] = log(w[0] / mu[1]);
  if (!maxent_newton(w, r, c, mmh, n0)) return false;
#pragma unroll
  for (int k = 0; k < 4; ++k) l[k] = c[k];
  return true;
}

#if FVM_MAXENT_WAVES > 0
#define FVM_MAXENT_ATTR __attribute__((amdgpu_waves_per_eu(FVM_MAXENT_WAVES)))
#else
#define FVM_MAXENT_ATTR
#endif

__global__ __launch_bounds__(kMeThreads) FVM_MAXENT_ATTR void maxent_source_kernel(
    StepArgs a, MaxEntRule r, MaxEntWarm wm) {
  const Spray m(a.m);
  bool cfl_fail;
  const double dt = launch_dt(a, cfl_fail);
  const double dte = cfl_fail ? 0.0 : dt;
  const double K = a.m.K, inv_theta = a.m.inv_theta;
  unsigned long long bx = 0, by = 0;
  const long long ncell = static_cast<long long>(a.g.nx) * a.g.ny;
  for (long long c = static_cast<long long>(blockIdx.x) * kMeThreads + threadIdx.x; c < ncell;
       c += static_cast<long long>(kMeThreads) * gridDim.x) {
    const int j = static_cast<int>(c / a.g.nx), i = static_cast<int>(c % a.g.nx);
    double* cell = a.wout + static_cast<size_t>(j) * a.g.ld + i;
    double w[6];
#pragma unroll
    for (int v = 0; v < 6; ++v) w[v] = cell[v * a.g.plane];
    const double m0 = w[0], m1 = w[1], m2 = w[2];
    // dt = 0 (a failed CFL check, a dry run) leaves the state as it is
    if (dte != 0.0 && m0 > 1e-300 && m1 > 1e-300 && m2 > 1e-300) {
      const size_t uc = ucell(a.g, j, i);
      const double ugx = a.ug[uc], ugy = a.ug[a.g.uplane + uc];
      // K = 0: no evaporation, and the closure is not needed
      double mmh = 0.0, n0 = 0.0;
      const size_t lc = static_cast<size_t>(j) * a.g.nx + i;
      const size_t lp = static_cast<size_t>(a.g.nx) * a.g.ny;
      double l[4] = {0.0, 0.0, 0.0, 0.0};
      if (wm.lam && wm.warm) {
#pragma unroll
        for (int k = 0; k < 4; ++k) l[k] = wm.lam[k * lp + lc];
      }
      const bool ok = K == 0.0 || maxent_closure(w, r, wm.warm != 0, l, mmh, n0);
      if (ok && K != 0.0 && wm.lam) {
#pragma unroll
        for (int k = 0; k < 4; ++k) wm.lam[k * lp + lc] = l[k];
      }
      if (ok) {
        const double r2 = 1.0 / m2;
        const double ux = w[4] * r2, uy = w[5] * r2;
        const double Km0 = K * m0;
        w[0] = fma(dte, -K * n0, m0);
        w[1] = fma(dte, -(0.5 * K) * mmh, m1);
        w[2] = fma(dte, -Km0, m2);
        w[3] = fma(dte, -(1.5 * K) * m1, w[3]);
        w[4] = fma(dte, fma(-Km0, ux, m0 * (ugx - ux) * inv_theta), w[4]);
        w[5] = fma(dte, fma(-Km0, uy, m0 * (ugy - uy) * inv_theta), w[5]);
      } else {
#pragma unroll
        for (int v = 0; v < 6; ++v) w[v] = __builtin_nan("");
      }
#pragma unroll
      for (int v = 0; v < 6; ++v) cell[v * a.g.plane] = w[v];
    }
    double sx, sy;
    m.speeds(w, sx, sy);
    bx = umax64(bx, bits(sx));
    by = umax64(by, bits(sy));
  }
  if (block_commit<kMeThreads / kWave>(bx, by, a.scr, gridDim.x) && threadIdx.x == 0) {
    if (cfl_fail) atomicOr(&a.scr->status, kStatusCfl);
    finalize_grid(a.scr, a.g, dte, true, nullptr);
  }
}

// Adjoint of the source step at the transported state, cell by cell:
// mu = lam + dt J_S(W*)^T lam (Sec. 2.2.2 eq. SourceTerm, Sec. 6.1 eq.
// Essadki). a.w holds W*, a.lam_in lam^{n+1}; mu goes to a.lam_out, which
// may be a.w itself (each thread reads its cell's W* before writing its mu).
// The closure rows: the multipliers l solve the dual's optimality
// conditions mu_{k+1}(l) = m_{k/2}, whose Jacobian in l is the moment
// Hessian H (H_kl = mu_{k+l+1}) and in m is -I, so dl/dm = H^{-1}; with
// n(S=0) = exp(l_0) and m_{-1/2} = int S^{-1/2} n dS,
//   dn0/dl = (n0, 0, 0, 0),   dm_{-1/2}/dl_k = int S^{-1/2} x^k n dS = mu_k,
// and the transposed rows are H^{-1} (-K lam_0 dn0/dl - K/2 lam_1 dm_{-1/2}/dl)
// (H is symmetric). Newton starts cold in every cell. A cell whose moments the
// closure cannot match gets NaN multipliers.
__global__ __launch_bounds__(kMeThreads) FVM_MAXENT_ATTR void maxent_adjoint_source_kernel(
    AdjointArgs a, const double* ug, MaxEntRule r) {
  const double dt = a.dts ? a.dts[a.k] : a.dt_arg;
  const double K = a.m.K, it = a.m.inv_theta;
  const long long ncell = static_cast<long long>(a.g.nx) * a.g.ny;
  for (long long c = static_cast<long long>(blockIdx.x) * kMeThreads + threadIdx.x; c < ncell;
       c += static_cast<long long>(kMeThreads) * gridDim.x) {
    const int j = static_cast<int>(c / a.g.nx), i = static_cast<int>(c % a.g.nx);
    const size_t at = static_cast<size_t>(j) * a.g.ld + i;
    double ws[6], lam[6], mu[6];
#pragma unroll
    for (int v = 0; v < 6; ++v) {
      ws[v] = a.w[v * a.g.plane + at];
      lam[v] = a.lam_in[v * a.g.plane + at];
      mu[v] = lam[v];
    }
    if (ws[0] > sadj::kVac && ws[1] > sadj::kVac && ws[2] > sadj::kVac) {
      const size_t uc = ucell(a.g, j, i);
      const double ugc[2] = {ug[uc], ug[a.g.uplane + uc]};
      double g[6];
      sadj::SprayAdj::source_rows(ws, lam, ugc, K, it, 1.0 / ws[2], g);
      if (K != 0.0) {
        double l[4] = {0.0, 0.0, 0.0, 0.0}, mmh, n0, m[8];
        bool ok = maxent_closure(ws, r, false, l, mmh, n0);
        double ya[4], yb[4];
        if (ok) {
          me_moments(l, r, m);
          // H y = rhs through the Newton direction solver (H d = -g)
          const double ra[4] = {K * lam[0] * n0, 0.0, 0.0, 0.0};
          const double rb[4] = {0.5 * K * lam[1] * m[0], 0.5 * K * lam[1] * m[1],
                                0.5 * K * lam[1] * m[2], 0.5 * K * lam[1] * m[3]};
          ok = me_direction(m, ra, ya) && me_direction(m, rb, yb);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) g[k] += ok ? ya[k] + yb[k] : __builtin_nan("");
      }
#pragma unroll
      for (int v = 0; v < 6; ++v) mu[v] = fma(dt, g[v], mu[v]);
    }
#pragma unroll
    for (int v = 0; v < 6; ++v) a.lam_out[v * a.g.plane + at] = mu[v];
  }
}

hipError_t launch_maxent_adjoint_source(const AdjointArgs& a, const double* ug, hipStream_t st);

// Gauss-Legendre rule of 8 points on [0, 1]: the roots of the Legendre
// polynomial P_8 (by Newton's method on the three-term recurrence, from the
// Chebyshev points) mapped from [-1, 1], weights 1 / ((1 - t^2) P_8'(t)^2).
static MaxEntRule gauss_legendre_8() {
  MaxEntRule r{};
  constexpr int n = 8;
  for (int i = 0; i < n; ++i) {
    double t = std::cos(M_PI * (i + 0.5) / n), dp = 1.0;
    for (int it = 0; it < 64; ++it) {
      double p0 = 1.0, p1 = t;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2 * k - 1) * t * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (t * p1 - p0) / (t * t - 1.0);
      const double step = p1 / dp;
      t -= step;
      if (std::fabs(step) < 1e-16) break;
    }
    r.x[i] = 0.5 * (t + 1.0);
    r.w[i] = 1.0 / ((1.0 - t * t) * dp * dp);
  }
  return r;
}

MaxEntLaunch maxent_launch(const StepArgs& a) {
  static const MaxEntRule rule = gauss_legendre_8();
  MaxEntLaunch l{};
  l.fn = reinterpret_cast<void*>(&maxent_source_kernel);
  const long long ncell = static_cast<long long>(a.g.nx) * a.g.ny;
  const long long blocks =
      std::min<long long>(kMeMaxBlocks, (ncell + kMeThreads - 1) / kMeThreads);
  l.grid = dim3(static_cast<unsigned>(blocks < 1 ? 1 : blocks));
  l.block = dim3(kMeThreads);
  l.rule = rule;
  return l;
}

hipError_t launch_maxent_source(const StepArgs& a, const MaxEntWarm& wm, hipStream_t st) {
  MaxEntLaunch l = maxent_launch(a);
  StepArgs copy = a;
  MaxEntWarm w = wm;
  void* args[] = {&copy, &l.rule, &w};
  return hipLaunchKernel(l.fn, l.grid, l.block, args, 0, st);
}

hipError_t launch_maxent_adjoint_source(const AdjointArgs& a, const double* ug, hipStream_t st) {
  static const MaxEntRule rule = gauss_legendre_8();
  const long long ncell = static_cast<long long>(a.g.nx) * a.g.ny;
  const long long blocks =
      std::min<long long>(kMeMaxBlocks, (ncell + kMeThreads - 1) / kMeThreads);
  hipLaunchKernelGGL(maxent_adjoint_source_kernel, dim3(static_cast<unsigned>(blocks < 1 ? 1 : blocks)),
                     dim3(kMeThreads), 0, st, a, ug, rule);
  return hipGetLastError();
}

}  // namespace fvm
