/*
 * fv_oracle.c -- plain, slow FP64 CPU oracle of the first-order finite-volume
 * time step (Essadki, Jung, Larat, Pelletier, Perrier, "A task-driven
 * implementation of a simple numerical solver for hyperbolic conservation
 * laws", CEMRACS 2016).
 *
 * TEST INFRASTRUCTURE ONLY. Nothing on the product path may link, load or
 * call this file: only the test-suite, the smoke check and the CPU-baseline leg
 * of the benchmark use it. It shares no code, header, table or constant with
 * the HIP library; the two only ever see the same seeded input arrays.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared (no fast-math), so
 * every floating-point operation below is one IEEE-754 double operation in the
 * order written (no fused multiply-add, no reassociation).
 *
 * Storage: structure-of-arrays W[v][j][i], x fastest, contiguous (pitch nx).
 * Cell (i,j) has centre ((i+1/2)dx, (j+1/2)dy), dx = lx/nx, dy = ly/ny.
 *
 * What each function follows:
 *   - the scheme itself: Sec. 2.2.1, eq. (VF_scheme), written in the residual
 *     form of Sec. 4.1 (eq. update, u += RHS) and Sec. 4.2 (eq. RHSFilling);
 *   - the Lax-Friedrichs (Rusanov) flux and its sigma: Sec. 2.2.1;
 *   - the CFL condition and the per-step check: Sec. 2.2.1 eq. (CFL_cond) and
 *     the checkTimeStep task of Sec. 4.2;
 *   - the source splitting: Sec. 2.2.2 eq. (SourceTerm);
 *   - the Euler system: Sec. 5 eq. (Euler);
 *   - the evaporating-spray moment system: Sec. 6.1 eqs. (Essadki), (Splitting);
 *   - the task decomposition (checkTimeStep, copyOverlaps, internalResiduals,
 *     borderResiduals, update) over NPartX x NPartY balanced subdomains with
 *     four one-cell overlap strips: Sec. 3.2 and Sec. 4.1-4.2.
 *
 * Readings where the paper is silent or garbled (each is also listed in the
 * design notes of the repository):
 *   R1 sign of RHS: eq. (RHSFilling) prints no minus sign, eq. (VF_scheme) and
 *      "u += RHS" need one: RHS = -[mux (F_{i+1/2}-F_{i-1/2}) + muy (G..-G..)].
 *   R2 adaptive time step: dt = C / (Sx/dx + Sy/dy) with Sx, Sy the largest
 *      x- and y-speeds over all cells (the 1-D form of eq. CFL_cond is kept
 *      as the check of fixed-dt steps).
 *   R3 the "direction n implicit" in the eigenvalues is read as the two axis
 *      normals: s_x = max_p |lambda_p(W,(1,0))|, s_y likewise.
 *   R4 linear advection uses the upwind flux a+ u_L + a- u_R, equal to the
 *      Lax-Friedrichs flux of the linear flux a u in exact arithmetic.
 *   R5 the spray transport uses the kinetic (pressureless) upwind flux
 *      F = W_L (u_L.n)+ + W_R (u_R.n)-, with u = q/m_{2/2}.
 *   R6 the spray closure (the paper reconstructs n(S) by entropy maximisation
 *      in a reference it cites, without giving the algorithm). Two closures:
 *      closure 0, a lognormal fit to (m_0, m_{1/2}, m_{2/2}) with n(S=0)
 *      read as the fitted density at S_eps; closure 1, the entropy maximiser
 *      itself, n(S) = exp(sum_k lambda_k S^{k/2}) on S in [0,1] matching the
 *      four moments, found by Newton's method on the convex dual with a
 *      backtracking line search and composite Gauss-Legendre quadrature in
 *      x = S^{1/2} (parity of this closure is pinned against an independent
 *      adaptive quadrature, not against the paper, which prints no values).
 *   R7 transmissive boundaries: a ghost cell equal to the boundary cell.
 *      Dirichlet boundaries (mentioned in Sec. 4.2 for the overlap of a
 *      subdomain at the domain's edge): the ghost cell holds a prescribed
 *      state, one constant state per side of the domain.
 *   R8 the adjoint (not in the paper) is the exact transpose of the
 *      implemented step with dt held fixed: the transport, and for the spray
 *      (lognormal closure only) the source at W* as well; max() follows the
 *      left argument on ties, d|x|/dx = +1 at x = 0, a clipped lognormal
 *      width is a constant, and every other branch is differentiated on the
 *      side it takes; a Dirichlet ghost state is a constant, so nothing
 *      flows back into it.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { ORC_ADV = 0, ORC_EULER = 1, ORC_SPRAY = 2 };
enum { ORC_PERIODIC = 0, ORC_TRANSMISSIVE = 1, ORC_DIRICHLET = 2 };
enum { ORC_WEST = 0, ORC_EAST = 1, ORC_SOUTH = 2, ORC_NORTH = 3 };
enum {
  ORC_OK = 0,
  ORC_EINVAL = -1,
  ORC_ECFL = -3,
  ORC_ENONFINITE = -4,
  ORC_EUNSUPPORTED = -5
};
#define ORC_MAXV 6
#define ORC_TINY 1e-300

typedef struct {
  int model, bc;
  int nx, ny, npx, npy;
  double lx, ly;
  double gamma, ax, ay;
  double K, theta, s_eps;
  double cfl, dt_max;
  double ghost[4][ORC_MAXV];  /* Dirichlet ghost states: west, east, south, north */
  int closure;                /* spray: 0 lognormal fit, 1 entropy maximiser (R6) */
} orc_params;

int orc_nvar(int model)
{
  switch (model) {
  case ORC_ADV: return 1;
  case ORC_EULER: return 4;
  case ORC_SPRAY: return 6;
  default: return 0;
  }
}

int orc_validate(const orc_params* P)
{
  if (!P) return ORC_EINVAL;
  if (orc_nvar(P->model) == 0) return ORC_EINVAL;
  if (P->bc != ORC_PERIODIC && P->bc != ORC_TRANSMISSIVE && P->bc != ORC_DIRICHLET)
    return ORC_EINVAL;
  if (P->nx < 1 || P->ny < 1 || P->npx < 1 || P->npy < 1) return ORC_EINVAL;
  /* balanced parts NxLoc = Nx/NPartX, NyLoc = Ny/NPartY (Sec. 3.2) */
  if (P->nx % P->npx != 0 || P->ny % P->npy != 0) return ORC_EINVAL;
  if (!(P->lx > 0) || !(P->ly > 0)) return ORC_EINVAL;
  if (P->model == ORC_EULER && !(P->gamma > 1)) return ORC_EINVAL;
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Pointwise physics                                                         */
/* ------------------------------------------------------------------------ */

/* Physical flux F(W).n along axis d (0 = x, 1 = y) and the largest
 * |eigenvalue| of dF.n/dW along that axis (reading R3). */
static void phys_flux(const orc_params* P, const double* w, int d, double* f,
                      double* s)
{
  if (P->model == ORC_ADV) {
    double a = (d == 0) ? P->ax : P->ay;
    f[0] = a * w[0];
    *s = fabs(a);
  } else if (P->model == ORC_EULER) {
    /* Sec. 5 eq. (Euler): W = (rho, rho u, rho v, rho E), perfect gas
     * p = (gamma-1) rho (E - (u^2+v^2)/2), eigenvalues u.n - c, u.n, u.n,
     * u.n + c with c^2 = gamma p / rho. */
    double r = w[0], ru = w[1], rv = w[2], e = w[3];
    double u = ru / r;
    double v = rv / r;
    double ke = 0.5 * (ru * u + rv * v);
    double p = (P->gamma - 1.0) * (e - ke);
    double c = sqrt(P->gamma * p / r);
    double un = (d == 0) ? u : v;
    f[0] = r * un;
    f[1] = ru * un;
    f[2] = rv * un;
    if (d == 0) f[1] = f[1] + p; else f[2] = f[2] + p;
    f[3] = (e + p) * un;
    *s = fabs(un) + c;
  } else {
    /* Sec. 6.1 eq. (Essadki): every component is transported with the
     * velocity u = (m_{2/2} u) / m_{2/2}. */
    double m2 = w[2];
    double un = 0.0;
    if (m2 > ORC_TINY) un = w[4 + d] / m2;
    for (int k = 0; k < 6; ++k) f[k] = w[k] * un;
    *s = fabs(un);
  }
}

/* Numerical flux F~(W_L, W_R, n) across a face with axis normal d. */
static void num_flux(const orc_params* P, const double* wl, const double* wr,
                     int d, double* f)
{
  if (P->model == ORC_ADV) {
    /* reading R4: upwind a+ u_L + a- u_R */
    double a = (d == 0) ? P->ax : P->ay;
    double ap = a > 0.0 ? a : 0.0;
    double am = a < 0.0 ? a : 0.0;
    f[0] = ap * wl[0] + am * wr[0];
  } else if (P->model == ORC_EULER) {
    /* Sec. 2.2.1: F~ = (F(W_L).n + F(W_R).n)/2 - sigma/2 (W_R - W_L),
     * sigma = max_p max(|lambda_p(W_L)|, |lambda_p(W_R)|). */
    double fl[4], fr[4], sl, sr;
    phys_flux(P, wl, d, fl, &sl);
    phys_flux(P, wr, d, fr, &sr);
    double sigma = sl >= sr ? sl : sr;
    for (int k = 0; k < 4; ++k)
      f[k] = 0.5 * (fl[k] + fr[k]) - 0.5 * sigma * (wr[k] - wl[k]);
  } else {
    /* reading R5: kinetic upwind flux of the pressureless transport */
    double ul = 0.0, ur = 0.0;
    if (wl[2] > ORC_TINY) ul = wl[4 + d] / wl[2];
    if (wr[2] > ORC_TINY) ur = wr[4 + d] / wr[2];
    double up = ul > 0.0 ? ul : 0.0;
    double um = ur < 0.0 ? ur : 0.0;
    for (int k = 0; k < 6; ++k) f[k] = wl[k] * up + wr[k] * um;
  }
}

/* Per-cell speeds for the time-step reduction. Returns 0 when the cell is
 * admissible; 1 when it is non-finite or non-physical (Euler: rho <= 0 or
 * p < 0; spray: a negative moment). */
static int cell_speeds(const orc_params* P, const double* w, double* sx,
                       double* sy)
{
  int nv = orc_nvar(P->model);
  for (int k = 0; k < nv; ++k)
    if (!isfinite(w[k])) return 1;
  double f[ORC_MAXV];
  phys_flux(P, w, 0, f, sx);
  phys_flux(P, w, 1, f, sy);
  if (!isfinite(*sx) || !isfinite(*sy)) return 1;
  if (P->model == ORC_EULER) {
    double r = w[0];
    double u = w[1] / r, v = w[2] / r;
    double p = (P->gamma - 1.0) * (w[3] - 0.5 * (w[1] * u + w[2] * v));
    if (!(r > 0.0) || !(p >= 0.0)) return 1;
  }
  if (P->model == ORC_SPRAY) {
    for (int k = 0; k < 4; ++k)
      if (w[k] < 0.0) return 1;
  }
  return 0;
}

/* The spray closure (reading R6). From (m_0, m_{1/2}, m_{2/2}) of a lognormal
 * n(S) = N0/(S s sqrt(2 pi)) exp(-(ln S - mu)^2 / (2 s^2)), whose fractional
 * moments are m_{k/2} = N0 exp(k mu/2 + k^2 s^2/8):
 *   L1 = ln(m_{1/2}/m_0) = mu/2 + s^2/8,  L2 = ln(m_{2/2}/m_0) = mu + s^2/2,
 *   s^2 = 4 (L2 - 2 L1),  mu = 2 L1 - s^2/4.
 * Returns m_{-1/2} and the density at S_eps. */
static void lognormal_closure(const orc_params* P, const double* w, double* mmh,
                          double* n0)
{
  double m0 = w[0], m1 = w[1], m2 = w[2];
  double L1 = log(m1 / m0);
  double L2 = log(m2 / m0);
  double s2 = 4.0 * (L2 - 2.0 * L1);
  if (s2 < 1e-8) s2 = 1e-8;
  double mu = 2.0 * L1 - s2 / 4.0;
  *mmh = m0 * exp(-mu / 2.0 + s2 / 8.0);
  double z = log(P->s_eps) - mu;
  *n0 = m0 / (P->s_eps * sqrt(2.0 * M_PI * s2)) * exp(-(z * z) / (2.0 * s2));
}

/* Gauss-Legendre rule of n points on [-1, 1]: the nodes are the roots of the
 * Legendre polynomial P_n, found by Newton's method from Tricomi's initial
 * guesses, with P_n and P_n' from the three-term recurrence
 * k P_k = (2k-1) z P_{k-1} - (k-1) P_{k-2}; the weights are
 * 2 / ((1 - z^2) P_n'(z)^2). */
static void gauss_legendre(int n, double* x, double* w)
{
  for (int i = 0; i < n; ++i) {
    double z = cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double pk = 1.0, pkm1 = 0.0;
      for (int k = 1; k <= n; ++k) {
        double pkm2 = pkm1;
        pkm1 = pk;
        pk = ((2.0 * k - 1.0) * z * pkm1 - (k - 1.0) * pkm2) / k;
      }
      dp = n * (z * pk - pkm1) / (z * z - 1.0);
      double dz = pk / dp;
      z -= dz;
      if (fabs(dz) <= 1e-17) break;
    }
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

/* Composite rule on x in [0, 1]: ME_PANELS panels of ME_NODES points. */
#define ME_PANELS 64
#define ME_NODES 16
#define ME_Q (ME_PANELS * ME_NODES)
static double me_x[ME_Q], me_w[ME_Q];
static int me_ready = 0;

static void maxent_rule(void)
{
  if (me_ready) return;
#pragma omp critical(orc_maxent_rule)
  {
    if (!me_ready) {
      double t[ME_NODES], v[ME_NODES];
      gauss_legendre(ME_NODES, t, v);
      for (int p = 0; p < ME_PANELS; ++p)
        for (int q = 0; q < ME_NODES; ++q) {
          double a = (double)p / ME_PANELS, h = 1.0 / ME_PANELS;
          me_x[p * ME_NODES + q] = a + 0.5 * h * (t[q] + 1.0);
          me_w[p * ME_NODES + q] = 0.5 * h * v[q];
        }
      me_ready = 1;
    }
  }
}

/* With S = x^2 (dS = 2x dx) and n(S) = exp(lambda_0 + lambda_1 x +
 * lambda_2 x^2 + lambda_3 x^3):
 *   mu[j+1] = int_0^1 S^{j/2} n(S) dS = 2 int_0^1 x^{j+1} n dx,  j = -1..6,
 * so mu[1..4] are the model's m_{0/2..3/2} and mu[0] = m_{-1/2}. */
static void maxent_moments(const double* lam, double* mu)
{
  for (int j = 0; j < 8; ++j) mu[j] = 0.0;
  for (int q = 0; q < ME_Q; ++q) {
    double x = me_x[q];
    double e = 2.0 * me_w[q] * exp(lam[0] + x * (lam[1] + x * (lam[2] + x * lam[3])));
    double xp = 1.0;
    for (int j = 0; j < 8; ++j) {
      mu[j] += e * xp;
      xp *= x;
    }
  }
}

/* Solves the 4x4 symmetric positive definite system H d = b (Cholesky);
 * returns 1 if H is not positive definite. */
static int spd_solve4(const double H[4][4], const double* b, double* d)
{
  double L[4][4] = {{0}};
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j <= i; ++j) {
      double s = H[i][j];
      for (int k = 0; k < j; ++k) s -= L[i][k] * L[j][k];
      if (i == j) {
        if (!(s > 0.0)) return 1;
        L[i][i] = sqrt(s);
      } else {
        L[i][j] = s / L[j][j];
      }
    }
  double y[4];
  for (int i = 0; i < 4; ++i) {
    double s = b[i];
    for (int k = 0; k < i; ++k) s -= L[i][k] * y[k];
    y[i] = s / L[i][i];
  }
  for (int i = 3; i >= 0; --i) {
    double s = y[i];
    for (int k = i + 1; k < 4; ++k) s -= L[k][i] * d[k];
    d[i] = s / L[i][i];
  }
  return 0;
}

/* The entropy maximiser of reading R6 (closure 1): the lambda minimising the
 * convex dual Phi(lambda) = int_0^1 n dS - sum_k lambda_k m_{k/2}, whose
 * gradient is the moment mismatch g_k = mu_k(lambda) - m_{k/2} and whose
 * Hessian is the moment matrix H_kl = mu_{k+l}. Newton steps from the normal
 * density in x that matches the mean and variance of x under n dS; while
 * the relative mismatch max_k |g_k|/m_{k/2} exceeds 1e-3 each step is cut
 * back until Phi decreases enough (Armijo), closer in the full step is
 * taken. Converged when the relative mismatch is <= 1e-14, or <= 1e-12 once
 * a step no longer halves it (the rounding floor of the quadrature sums).
 * Returns 0 and (lambda, m_{-1/2}, n(S=0) = exp(lambda_0)), or 1 if the
 * moments are not realisable or Newton does not converge. */
int orc_maxent(const double* m, double* lam_out, double* mmh, double* n0)
{
  maxent_rule();
  if (!(m[0] > ORC_TINY)) return 1;
  double a = m[1] / m[0], var = m[2] / m[0] - a * a;
  if (!(var > 0.0)) return 1;
  double lam[4] = {0.0, a / var, -0.5 / var, 0.0}, mu[8];
  maxent_moments(lam, mu);
  if (!(mu[1] > 0.0)) return 1;
  lam[0] = log(m[0] / mu[1]);
  maxent_moments(lam, mu);
  int ok = 0;
  double prev = INFINITY;
  for (int it = 0; it < 200; ++it) {
    double g[4], rel = 0.0;
    for (int k = 0; k < 4; ++k) {
      g[k] = mu[k + 1] - m[k];
      double r = fabs(g[k]) / m[k];
      if (!(r <= rel)) rel = r; /* NaN-sticky */
    }
    if (!(rel == rel)) return 1;
    if (rel <= 1e-14 || (rel <= 1e-12 && rel > 0.5 * prev)) {
      ok = 1;
      break;
    }
    prev = rel;
    double H[4][4], d[4], b[4];
    for (int k = 0; k < 4; ++k) {
      b[k] = -g[k];
      for (int l = 0; l < 4; ++l) H[k][l] = mu[k + l + 1];
    }
    if (spd_solve4(H, b, d)) return 1;
    double t = 1.0, trial[4], mt[8];
    if (rel > 1e-3) {
      double phi = mu[1], slope = 0.0;
      for (int k = 0; k < 4; ++k) {
        phi -= lam[k] * m[k];
        slope += g[k] * d[k];
      }
      int accepted = 0;
      for (int ls = 0; ls < 60 && !accepted; ++ls) {
        for (int k = 0; k < 4; ++k) trial[k] = lam[k] + t * d[k];
        maxent_moments(trial, mt);
        double pt = mt[1];
        for (int k = 0; k < 4; ++k) pt -= trial[k] * m[k];
        if (pt <= phi + 1e-4 * t * slope)
          accepted = 1;
        else
          t *= 0.5;
      }
      if (!accepted) return 1;
    } else {
      for (int k = 0; k < 4; ++k) trial[k] = lam[k] + d[k];
      maxent_moments(trial, mt);
    }
    for (int k = 0; k < 4; ++k) lam[k] = trial[k];
    for (int j = 0; j < 8; ++j) mu[j] = mt[j];
  }
  if (!ok) return 1;
  for (int k = 0; k < 4; ++k) lam_out[k] = lam[k];
  *mmh = mu[0];
  *n0 = exp(lam[0]);
  return 0;
}

/* m_{-1/2} and n(S=0) from the closure the parameters select; returns 1 if
 * the entropy maximiser fails. */
static int spray_closure(const orc_params* P, const double* w, double* mmh,
                         double* n0)
{
  if (P->closure == 1) {
    double lam[4];
    return orc_maxent(w, lam, mmh, n0);
  }
  lognormal_closure(P, w, mmh, n0);
  return 0;
}

/* Source S(W) of Sec. 6.1 eq. (Essadki): evaporation on the four moments and
 * on the momentum, drag m_0 (u_g - u)/theta on the momentum. */
static void spray_source(const orc_params* P, const double* w,
                         const double* ug, double* S)
{
  double m0 = w[0], m1 = w[1], m2 = w[2];
  for (int k = 0; k < 6; ++k) S[k] = 0.0;
  if (!(m0 > ORC_TINY) || !(m1 > ORC_TINY) || !(m2 > ORC_TINY)) return;
  double ux = w[4] / m2, uy = w[5] / m2;
  /* with K = 0 the evaporation terms vanish and the closure is not needed */
  double mmh = 0.0, n0 = 0.0;
  if (P->K != 0.0 && spray_closure(P, w, &mmh, &n0)) {
    /* moments the entropy maximiser cannot match: the cell becomes
     * non-finite, which the next speed check reports */
    for (int k = 0; k < 6; ++k) S[k] = NAN;
    return;
  }
  double K = P->K;
  S[0] = -K * n0;
  S[1] = -(K / 2.0) * mmh;
  S[2] = -K * m0;
  S[3] = -(1.5 * K) * m1;
  S[4] = -K * m0 * ux + m0 * (ug[0] - ux) / P->theta;
  S[5] = -K * m0 * uy + m0 * (ug[1] - uy) / P->theta;
}

/* ------------------------------------------------------------------------ */
/* Exported pointwise helpers (used by the pins in the test-suite)           */
/* ------------------------------------------------------------------------ */

/* w: nvar values of one state; f: nvar values. */
void orc_phys_flux(const orc_params* P, const double* w, int d, double* f,
                   double* s)
{
  phys_flux(P, w, d, f, s);
}

void orc_num_flux(const orc_params* P, const double* wl, const double* wr,
                  int d, double* f)
{
  num_flux(P, wl, wr, d, f);
}

int orc_cell_speeds(const orc_params* P, const double* w, double* sx,
                    double* sy)
{
  return cell_speeds(P, w, sx, sy);
}

int orc_spray_closure(const orc_params* P, const double* w, double* mmh,
                      double* n0)
{
  return spray_closure(P, w, mmh, n0);
}

void orc_spray_source(const orc_params* P, const double* w, const double* ug,
                      double* S)
{
  spray_source(P, w, ug, S);
}

/* ------------------------------------------------------------------------ */
/* The partitioned solver: subdomains with overlap strips (Sec. 3.2, 4.1)    */
/* ------------------------------------------------------------------------ */

typedef struct {
  int nxl, nyl;              /* NxLoc, NyLoc */
  double* u;                 /* uLoc: nv x nyl x nxl */
  double* rhs;               /* RHS:  nv x nyl x nxl */
  double* ovE;               /* ovlpE: nv x nyl (east neighbour's west column) */
  double* ovW;               /* ovlpW: nv x nyl */
  double* ovN;               /* ovlpN: nv x nxl (north neighbour's south row) */
  double* ovS;               /* ovlpS: nv x nxl */
  double* fx;                /* x-face fluxes: nv x nyl x (nxl+1) */
  double* fy;                /* y-face fluxes: nv x (nyl+1) x nxl */
  double sx, sy;             /* local speed maxima (checkTimeStep) */
  int bad;                   /* a non-admissible cell was seen */
} orc_part;

typedef struct {
  orc_params P;
  int nv, nparts;
  orc_part* part;
  const double* ug;          /* spray gas velocity, 2 x ny x nx, or NULL */
} orc_solver;

#define U_(p, v, j, i) ((p)->u[((size_t)(v) * (p)->nyl + (j)) * (p)->nxl + (i)])
#define R_(p, v, j, i) ((p)->rhs[((size_t)(v) * (p)->nyl + (j)) * (p)->nxl + (i)])

static void solver_free(orc_solver* S)
{
  if (!S->part) return;
  for (int q = 0; q < S->nparts; ++q) {
    orc_part* p = &S->part[q];
    free(p->u); free(p->rhs); free(p->ovE); free(p->ovW);
    free(p->ovN); free(p->ovS); free(p->fx); free(p->fy);
  }
  free(S->part);
  S->part = NULL;
}

static int solver_init(orc_solver* S, const orc_params* P, const double* ug)
{
  memset(S, 0, sizeof(*S));
  S->P = *P;
  S->nv = orc_nvar(P->model);
  S->nparts = P->npx * P->npy;
  S->ug = ug;
  S->part = (orc_part*)calloc((size_t)S->nparts, sizeof(orc_part));
  if (!S->part) return ORC_EINVAL;
  int nxl = P->nx / P->npx, nyl = P->ny / P->npy, nv = S->nv;
  for (int q = 0; q < S->nparts; ++q) {
    orc_part* p = &S->part[q];
    p->nxl = nxl;
    p->nyl = nyl;
    p->u = (double*)malloc(sizeof(double) * nv * nxl * nyl);
    p->rhs = (double*)malloc(sizeof(double) * nv * nxl * nyl);
    p->ovE = (double*)malloc(sizeof(double) * nv * nyl);
    p->ovW = (double*)malloc(sizeof(double) * nv * nyl);
    p->ovN = (double*)malloc(sizeof(double) * nv * nxl);
    p->ovS = (double*)malloc(sizeof(double) * nv * nxl);
    p->fx = (double*)malloc(sizeof(double) * nv * nyl * (nxl + 1));
    p->fy = (double*)malloc(sizeof(double) * nv * (nyl + 1) * nxl);
    if (!p->u || !p->rhs || !p->ovE || !p->ovW || !p->ovN || !p->ovS ||
        !p->fx || !p->fy) {
      solver_free(S);
      return ORC_EINVAL;
    }
  }
  return ORC_OK;
}

/* subdomain (px,py) -> index; px fastest */
static int part_id(const orc_params* P, int px, int py)
{
  return py * P->npx + px;
}

/* copy the global array into the per-subdomain uLoc handles */
static void scatter(orc_solver* S, const double* W)
{
  const orc_params* P = &S->P;
  for (int q = 0; q < S->nparts; ++q) {
    orc_part* p = &S->part[q];
    int px = q % P->npx, py = q / P->npx;
    for (int v = 0; v < S->nv; ++v)
      for (int j = 0; j < p->nyl; ++j)
        for (int i = 0; i < p->nxl; ++i)
          U_(p, v, j, i) = W[((size_t)v * P->ny + (size_t)py * p->nyl + j) * P->nx +
                             (size_t)px * p->nxl + i];
  }
}

static void gather(const orc_solver* S, double* W)
{
  const orc_params* P = &S->P;
  for (int q = 0; q < S->nparts; ++q) {
    const orc_part* p = &S->part[q];
    int px = q % P->npx, py = q / P->npx;
    for (int v = 0; v < S->nv; ++v)
      for (int j = 0; j < p->nyl; ++j)
        for (int i = 0; i < p->nxl; ++i)
          W[((size_t)v * P->ny + (size_t)py * p->nyl + j) * P->nx +
            (size_t)px * p->nxl + i] = U_(p, v, j, i);
  }
}

/* checkTimeStep: the largest characteristic speeds within one subdomain. */
static void task_check_time_step(const orc_solver* S, orc_part* p)
{
  double w[ORC_MAXV];
  p->sx = 0.0;
  p->sy = 0.0;
  p->bad = 0;
  for (int j = 0; j < p->nyl; ++j)
    for (int i = 0; i < p->nxl; ++i) {
      for (int v = 0; v < S->nv; ++v) w[v] = U_(p, v, j, i);
      double sx, sy;
      if (cell_speeds(&S->P, w, &sx, &sy)) {
        p->bad = 1;
        continue;
      }
      if (sx > p->sx) p->sx = sx;
      if (sy > p->sy) p->sy = sy;
    }
}

/* copyOverlaps: subdomain (px,py) fills its neighbours' overlap strips.
 * Its north row goes to ovlpS of the north neighbour, its south row to ovlpN
 * of the south neighbour, its east column to ovlpW of the east neighbour and
 * its west column to ovlpE of the west neighbour (Sec. 4.2). On a physical
 * transmissive boundary the subdomain fills its own strip with its own
 * border (ghost = boundary cell, reading R7), on a Dirichlet boundary with
 * the side's prescribed state; on a periodic boundary the neighbour wraps
 * around (it may be the subdomain itself). */
static void task_copy_overlaps(orc_solver* S, int q)
{
  const orc_params* P = &S->P;
  orc_part* p = &S->part[q];
  int px = q % P->npx, py = q / P->npx;
  int nv = S->nv, nxl = p->nxl, nyl = p->nyl;
  int per = (P->bc == ORC_PERIODIC);
  int dir = (P->bc == ORC_DIRICHLET);

  /* north row -> ovlpS of the north neighbour */
  if (py + 1 < P->npy || per) {
    orc_part* nb = &S->part[part_id(P, px, (py + 1) % P->npy)];
    for (int v = 0; v < nv; ++v)
      for (int i = 0; i < nxl; ++i) nb->ovS[v * nxl + i] = U_(p, v, nyl - 1, i);
  } else {
    for (int v = 0; v < nv; ++v)
      for (int i = 0; i < nxl; ++i)
        p->ovN[v * nxl + i] = dir ? P->ghost[ORC_NORTH][v] : U_(p, v, nyl - 1, i);
  }
  /* south row -> ovlpN of the south neighbour */
  if (py > 0 || per) {
    orc_part* nb = &S->part[part_id(P, px, (py + P->npy - 1) % P->npy)];
    for (int v = 0; v < nv; ++v)
      for (int i = 0; i < nxl; ++i) nb->ovN[v * nxl + i] = U_(p, v, 0, i);
  } else {
    for (int v = 0; v < nv; ++v)
      for (int i = 0; i < nxl; ++i)
        p->ovS[v * nxl + i] = dir ? P->ghost[ORC_SOUTH][v] : U_(p, v, 0, i);
  }
  /* east column -> ovlpW of the east neighbour */
  if (px + 1 < P->npx || per) {
    orc_part* nb = &S->part[part_id(P, (px + 1) % P->npx, py)];
    for (int v = 0; v < nv; ++v)
      for (int j = 0; j < nyl; ++j) nb->ovW[v * nyl + j] = U_(p, v, j, nxl - 1);
  } else {
    for (int v = 0; v < nv; ++v)
      for (int j = 0; j < nyl; ++j)
        p->ovE[v * nyl + j] = dir ? P->ghost[ORC_EAST][v] : U_(p, v, j, nxl - 1);
  }
  /* west column -> ovlpE of the west neighbour */
  if (px > 0 || per) {
    orc_part* nb = &S->part[part_id(P, (px + P->npx - 1) % P->npx, py)];
    for (int v = 0; v < nv; ++v)
      for (int j = 0; j < nyl; ++j) nb->ovE[v * nyl + j] = U_(p, v, j, 0);
  } else {
    for (int v = 0; v < nv; ++v)
      for (int j = 0; j < nyl; ++j)
        p->ovW[v * nyl + j] = dir ? P->ghost[ORC_WEST][v] : U_(p, v, j, 0);
  }
}

#define FX_(p, v, j, f) ((p)->fx[((size_t)(v) * (p)->nyl + (j)) * ((p)->nxl + 1) + (f)])
#define FY_(p, v, f, i) ((p)->fy[((size_t)(v) * ((p)->nyl + 1) + (f)) * (p)->nxl + (i)])

/* RHS of one cell from its four face fluxes (reading R1):
 * RHS = -(mux (F_E - F_W) + muy (G_N - G_S)). */
static void cell_rhs(const orc_solver* S, orc_part* p, int j, int i,
                     double mux, double muy)
{
  for (int v = 0; v < S->nv; ++v) {
    double t = mux * (FX_(p, v, j, i + 1) - FX_(p, v, j, i)) +
               muy * (FY_(p, v, j + 1, i) - FY_(p, v, j, i));
    R_(p, v, j, i) = -t;
  }
}

/* internalResiduals: fluxes at every face with both cells inside the
 * subdomain (each face once), then the RHS of every cell whose four faces
 * are all interior. */
static void task_internal_residuals(orc_solver* S, orc_part* p, double mux,
                                    double muy)
{
  double wl[ORC_MAXV], wr[ORC_MAXV], f[ORC_MAXV];
  int nv = S->nv;
  for (int j = 0; j < p->nyl; ++j)
    for (int i = 0; i + 1 < p->nxl; ++i) {
      for (int v = 0; v < nv; ++v) {
        wl[v] = U_(p, v, j, i);
        wr[v] = U_(p, v, j, i + 1);
      }
      num_flux(&S->P, wl, wr, 0, f);
      for (int v = 0; v < nv; ++v) FX_(p, v, j, i + 1) = f[v];
    }
  for (int j = 0; j + 1 < p->nyl; ++j)
    for (int i = 0; i < p->nxl; ++i) {
      for (int v = 0; v < nv; ++v) {
        wl[v] = U_(p, v, j, i);
        wr[v] = U_(p, v, j + 1, i);
      }
      num_flux(&S->P, wl, wr, 1, f);
      for (int v = 0; v < nv; ++v) FY_(p, v, j + 1, i) = f[v];
    }
  for (int j = 1; j + 1 < p->nyl; ++j)
    for (int i = 1; i + 1 < p->nxl; ++i) cell_rhs(S, p, j, i, mux, muy);
}

/* borderResiduals: the fluxes between the overlap strips and the border
 * cells, then the RHS of the border ring. */
static void task_border_residuals(orc_solver* S, orc_part* p, double mux,
                                  double muy)
{
  double wl[ORC_MAXV], wr[ORC_MAXV], f[ORC_MAXV];
  int nv = S->nv, nxl = p->nxl, nyl = p->nyl;
  for (int j = 0; j < nyl; ++j) {
    /* west face: ovlpW | cell 0 */
    for (int v = 0; v < nv; ++v) {
      wl[v] = p->ovW[v * nyl + j];
      wr[v] = U_(p, v, j, 0);
    }
    num_flux(&S->P, wl, wr, 0, f);
    for (int v = 0; v < nv; ++v) FX_(p, v, j, 0) = f[v];
    /* east face: cell nxl-1 | ovlpE */
    for (int v = 0; v < nv; ++v) {
      wl[v] = U_(p, v, j, nxl - 1);
      wr[v] = p->ovE[v * nyl + j];
    }
    num_flux(&S->P, wl, wr, 0, f);
    for (int v = 0; v < nv; ++v) FX_(p, v, j, nxl) = f[v];
  }
  for (int i = 0; i < nxl; ++i) {
    /* south face: ovlpS | row 0 */
    for (int v = 0; v < nv; ++v) {
      wl[v] = p->ovS[v * nxl + i];
      wr[v] = U_(p, v, 0, i);
    }
    num_flux(&S->P, wl, wr, 1, f);
    for (int v = 0; v < nv; ++v) FY_(p, v, 0, i) = f[v];
    /* north face: row nyl-1 | ovlpN */
    for (int v = 0; v < nv; ++v) {
      wl[v] = U_(p, v, nyl - 1, i);
      wr[v] = p->ovN[v * nxl + i];
    }
    num_flux(&S->P, wl, wr, 1, f);
    for (int v = 0; v < nv; ++v) FY_(p, v, nyl, i) = f[v];
  }
  for (int j = 0; j < nyl; ++j)
    for (int i = 0; i < nxl; ++i)
      if (j == 0 || j == nyl - 1 || i == 0 || i == nxl - 1)
        cell_rhs(S, p, j, i, mux, muy);
}

/* update: u += RHS (Sec. 4.1 eq. update). */
static void task_update(orc_solver* S, orc_part* p)
{
  size_t n = (size_t)S->nv * p->nxl * p->nyl;
  for (size_t k = 0; k < n; ++k) p->u[k] = p->u[k] + p->rhs[k];
}

/* source: W^{n+1} = W* + dt S(W*) cell by cell (Sec. 2.2.2 eq. SourceTerm). */
static void task_source(orc_solver* S, orc_part* p, int q, double dt)
{
  const orc_params* P = &S->P;
  int px = q % P->npx, py = q / P->npx;
  double w[ORC_MAXV], g[2], src[ORC_MAXV];
  for (int j = 0; j < p->nyl; ++j)
    for (int i = 0; i < p->nxl; ++i) {
      size_t gi = (size_t)(py * p->nyl + j) * P->nx + (size_t)px * p->nxl + i;
      for (int v = 0; v < 6; ++v) w[v] = U_(p, v, j, i);
      g[0] = S->ug[gi];
      g[1] = S->ug[(size_t)P->nx * P->ny + gi];
      spray_source(P, w, g, src);
      for (int v = 0; v < 6; ++v) U_(p, v, j, i) = w[v] + dt * src[v];
    }
}

/* Global speed maxima over all subdomains; returns ORC_ENONFINITE if a cell
 * is not admissible. */
static int all_speeds(orc_solver* S, double* Sx, double* Sy)
{
  int q;
#pragma omp parallel for schedule(dynamic, 1)
  for (q = 0; q < S->nparts; ++q) task_check_time_step(S, &S->part[q]);
  double mx = 0.0, my = 0.0;
  int bad = 0;
  for (q = 0; q < S->nparts; ++q) {
    if (S->part[q].bad) bad = 1;
    if (S->part[q].sx > mx) mx = S->part[q].sx;
    if (S->part[q].sy > my) my = S->part[q].sy;
  }
  *Sx = mx;
  *Sy = my;
  return bad ? ORC_ENONFINITE : ORC_OK;
}

/* reading R2 */
static int dt_from_speeds(const orc_params* P, double Sx, double Sy,
                          double* dt)
{
  double dx = P->lx / P->nx, dy = P->ly / P->ny;
  if (Sx == 0.0 && Sy == 0.0) {
    if (!(P->dt_max > 0.0)) return ORC_EINVAL;
    *dt = P->dt_max;
    return ORC_OK;
  }
  *dt = P->cfl / (Sx / dx + Sy / dy);
  return ORC_OK;
}

/* One time step of the subdomain tasks with a given dt. */
static void step_tasks(orc_solver* S, double dt)
{
  const orc_params* P = &S->P;
  double mux = dt / (P->lx / P->nx), muy = dt / (P->ly / P->ny);
  int q;
#pragma omp parallel for schedule(dynamic, 1)
  for (q = 0; q < S->nparts; ++q) task_copy_overlaps(S, q);
#pragma omp parallel for schedule(dynamic, 1)
  for (q = 0; q < S->nparts; ++q) task_internal_residuals(S, &S->part[q], mux, muy);
#pragma omp parallel for schedule(dynamic, 1)
  for (q = 0; q < S->nparts; ++q) task_border_residuals(S, &S->part[q], mux, muy);
#pragma omp parallel for schedule(dynamic, 1)
  for (q = 0; q < S->nparts; ++q) task_update(S, &S->part[q]);
  if (P->model == ORC_SPRAY) {
#pragma omp parallel for schedule(dynamic, 1)
    for (q = 0; q < S->nparts; ++q) task_source(S, &S->part[q], q, dt);
  }
}

/* ------------------------------------------------------------------------ */
/* Exported drivers                                                          */
/* ------------------------------------------------------------------------ */

void orc_set_threads(int n)
{
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int orc_get_threads(void)
{
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* checkTimeStep over the whole grid: speed maxima and the adaptive dt. */
int orc_cfl(const orc_params* P, const double* W, double* Sx, double* Sy,
            double* dt)
{
  int rc = orc_validate(P);
  if (rc) return rc;
  orc_solver S;
  if (solver_init(&S, P, NULL)) return ORC_EINVAL;
  scatter(&S, W);
  rc = all_speeds(&S, Sx, Sy);
  if (rc == ORC_OK) rc = dt_from_speeds(P, *Sx, *Sy, dt);
  solver_free(&S);
  return rc;
}

/* nsteps adaptive steps in place: each step runs checkTimeStep, takes
 * dt = C/(Sx/dx + Sy/dy), then the subdomain tasks. dts (nullable) receives
 * the nsteps time steps. */
int orc_run(const orc_params* P, double* W, const double* ug, int nsteps,
            double* dts)
{
  int rc = orc_validate(P);
  if (rc) return rc;
  if (P->model == ORC_SPRAY && !ug) return ORC_EINVAL;
  if (nsteps < 0) return ORC_EINVAL;
  orc_solver S;
  if (solver_init(&S, P, ug)) return ORC_EINVAL;
  scatter(&S, W);
  for (int n = 0; n < nsteps && rc == ORC_OK; ++n) {
    double Sx, Sy, dt;
    rc = all_speeds(&S, &Sx, &Sy);
    if (rc) break;
    rc = dt_from_speeds(P, Sx, Sy, &dt);
    if (rc) break;
    if (dts) dts[n] = dt;
    step_tasks(&S, dt);
  }
  gather(&S, W);
  solver_free(&S);
  return rc;
}

/* nsteps steps in place with the given time steps (no CFL logic). */
int orc_run_dts(const orc_params* P, double* W, const double* ug, int nsteps,
                const double* dts)
{
  int rc = orc_validate(P);
  if (rc) return rc;
  if (P->model == ORC_SPRAY && !ug) return ORC_EINVAL;
  if (nsteps < 0 || (nsteps > 0 && !dts)) return ORC_EINVAL;
  orc_solver S;
  if (solver_init(&S, P, ug)) return ORC_EINVAL;
  scatter(&S, W);
  for (int n = 0; n < nsteps; ++n) step_tasks(&S, dts[n]);
  gather(&S, W);
  solver_free(&S);
  return ORC_OK;
}

/* One step with a fixed dt, checked as in the checkTimeStep task:
 * dt * max_cells max_p |lambda_p| <= min(dx, dy) (eq. CFL_cond). On failure
 * the state is left unchanged and ORC_ECFL returned. */
int orc_step_fixed(const orc_params* P, double* W, const double* ug, double dt)
{
  int rc = orc_validate(P);
  if (rc) return rc;
  if (!(dt > 0.0) || !isfinite(dt)) return ORC_EINVAL;
  if (P->model == ORC_SPRAY && !ug) return ORC_EINVAL;
  orc_solver S;
  if (solver_init(&S, P, ug)) return ORC_EINVAL;
  scatter(&S, W);
  double Sx, Sy;
  rc = all_speeds(&S, &Sx, &Sy);
  if (rc == ORC_OK) {
    double dx = P->lx / P->nx, dy = P->ly / P->ny;
    double smax = Sx > Sy ? Sx : Sy;
    double hmin = dx < dy ? dx : dy;
    if (dt * smax > hmin) rc = ORC_ECFL;
  }
  if (rc == ORC_OK) {
    step_tasks(&S, dt);
    gather(&S, W);
  }
  solver_free(&S);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Adjoint of the transport step (reading R8)                                 */
/* ------------------------------------------------------------------------ */

/* A = d(F(W).n)/dW for the Euler flux along axis d, written out row by row. */
static void euler_flux_jacobian(const orc_params* P, const double* w, int d,
                                double A[4][4])
{
  double g = P->gamma;
  double r = w[0], u = w[1] / r, v = w[2] / r, e = w[3];
  double q2 = u * u + v * v;
  double p = (g - 1.0) * (e - 0.5 * r * q2);
  double H = (e + p) / r;
  /* dp/dW */
  double dp[4] = {(g - 1.0) * 0.5 * q2, -(g - 1.0) * u, -(g - 1.0) * v, g - 1.0};
  double un = d == 0 ? u : v;
  /* dun/dW */
  double dun[4] = {-un / r, d == 0 ? 1.0 / r : 0.0, d == 0 ? 0.0 : 1.0 / r, 0.0};
  /* row 0: rho un = W[1+d] */
  for (int l = 0; l < 4; ++l) A[0][l] = 0.0;
  A[0][1 + d] = 1.0;
  /* rows 1,2: W[k] un + p n_k */
  for (int k = 1; k <= 2; ++k)
    for (int l = 0; l < 4; ++l) {
      double a = w[k] * dun[l];
      if (l == k) a = a + un;
      if (k == 1 + d) a = a + dp[l];
      A[k][l] = a;
    }
  /* row 3: (e + p) un */
  for (int l = 0; l < 4; ++l) {
    double de = (l == 3) ? 1.0 : 0.0;
    A[3][l] = (de + dp[l]) * un + (e + p) * dun[l];
  }
  (void)H;
}

/* gradient of s = |un| + c with respect to W (Euler) */
static void euler_speed_gradient(const orc_params* P, const double* w, int d,
                                 double gs[4])
{
  double g = P->gamma;
  double r = w[0], u = w[1] / r, v = w[2] / r, e = w[3];
  double q2 = u * u + v * v;
  double p = (g - 1.0) * (e - 0.5 * r * q2);
  double c = sqrt(g * p / r);
  double un = d == 0 ? u : v;
  double sgn = un >= 0.0 ? 1.0 : -1.0;
  double dp[4] = {(g - 1.0) * 0.5 * q2, -(g - 1.0) * u, -(g - 1.0) * v, g - 1.0};
  double dun[4] = {-un / r, d == 0 ? 1.0 / r : 0.0, d == 0 ? 0.0 : 1.0 / r, 0.0};
  /* c^2 = g p / r  =>  dc = g/(2 c r) (dp - p/r drho) */
  for (int l = 0; l < 4; ++l) {
    double dpl = dp[l];
    if (l == 0) dpl = dpl - p / r;
    gs[l] = sgn * dun[l] + g / (2.0 * c * r) * dpl;
  }
}

/* Jacobians of the kinetic upwind flux (reading R5) with respect to its left
 * and right states: F = W_L up + W_R um with up = max(u_L.n, 0),
 * um = min(u_R.n, 0) and u.n = W[4+d] / W[2]. The branch taken decides the
 * derivative (at u.n = 0 both are the zero branch); below the vacuum
 * threshold u.n is the constant 0. */
static void spray_flux_jacobians(const double* wl, const double* wr, int d,
                                 double JL[ORC_MAXV][ORC_MAXV],
                                 double JR[ORC_MAXV][ORC_MAXV])
{
  double ul = 0.0, ur = 0.0, gl[6] = {0}, gr[6] = {0};
  if (wl[2] > ORC_TINY) {
    ul = wl[4 + d] / wl[2];
    gl[2] = -ul / wl[2];
    gl[4 + d] = 1.0 / wl[2];
  }
  if (wr[2] > ORC_TINY) {
    ur = wr[4 + d] / wr[2];
    gr[2] = -ur / wr[2];
    gr[4 + d] = 1.0 / wr[2];
  }
  int pos = ul > 0.0, neg = ur < 0.0;
  double up = pos ? ul : 0.0, um = neg ? ur : 0.0;
  for (int k = 0; k < 6; ++k)
    for (int l = 0; l < 6; ++l) {
      double id = (k == l) ? 1.0 : 0.0;
      JL[k][l] = id * up + (pos ? wl[k] * gl[l] : 0.0);
      JR[k][l] = id * um + (neg ? wr[k] * gr[l] : 0.0);
    }
}

/* Jacobians of the numerical flux with respect to its left and right states. */
static void num_flux_jacobians(const orc_params* P, const double* wl,
                               const double* wr, int d,
                               double JL[ORC_MAXV][ORC_MAXV],
                               double JR[ORC_MAXV][ORC_MAXV])
{
  if (P->model == ORC_ADV) {
    double a = (d == 0) ? P->ax : P->ay;
    JL[0][0] = a > 0.0 ? a : 0.0;
    JR[0][0] = a < 0.0 ? a : 0.0;
    return;
  }
  if (P->model == ORC_SPRAY) {
    spray_flux_jacobians(wl, wr, d, JL, JR);
    return;
  }
  double AL[4][4], AR[4][4], gl[4], gr[4], f[4], sl, sr;
  euler_flux_jacobian(P, wl, d, AL);
  euler_flux_jacobian(P, wr, d, AR);
  phys_flux(P, wl, d, f, &sl);
  phys_flux(P, wr, d, f, &sr);
  euler_speed_gradient(P, wl, d, gl);
  euler_speed_gradient(P, wr, d, gr);
  int left = sl >= sr;
  double sigma = left ? sl : sr;
  for (int k = 0; k < 4; ++k)
    for (int l = 0; l < 4; ++l) {
      double dw = wr[k] - wl[k];
      double id = (k == l) ? 1.0 : 0.0;
      JL[k][l] = 0.5 * AL[k][l] + 0.5 * sigma * id - 0.5 * dw * (left ? gl[l] : 0.0);
      JR[k][l] = 0.5 * AR[k][l] - 0.5 * sigma * id - 0.5 * dw * (left ? 0.0 : gr[l]);
    }
}

/* J = dS/dW of the spray source (Sec. 6.1 eq. Essadki), differentiated by
 * hand; for the entropy-maximising closure (Sec. 6.2) the two closure rows
 * follow from the optimality conditions of its dual (below); with the
 * lognormal closure (reading R6):
 * L1 = ln(m_{1/2}/m_0), L2 = ln(m_{2/2}/m_0), s^2 = 4 (L2 - 2 L1) (a constant
 * where it is clipped at 1e-8), mu = 2 L1 - s^2/4,
 *   d ln m_{-1/2} = dm_0/m_0 - dmu/2 + ds^2/8,
 *   d ln n(S_eps) = dm_0/m_0 - ds^2/(2 s^2) + z dmu/s^2 + z^2 ds^2/(2 s^4),
 * z = ln S_eps - mu; the momentum rows follow from u = q/m_{2/2}. Zero where
 * the source is switched off (a moment at or below the vacuum threshold). */
static void spray_source_jacobian(const orc_params* P, const double* w,
                                  const double* ug, double J[6][6])
{
  for (int k = 0; k < 6; ++k)
    for (int l = 0; l < 6; ++l) J[k][l] = 0.0;
  double m0 = w[0], m1 = w[1], m2 = w[2];
  if (!(m0 > ORC_TINY) || !(m1 > ORC_TINY) || !(m2 > ORC_TINY)) return;
  double K = P->K, it = 1.0 / P->theta;
  double u[2] = {w[4] / m2, w[5] / m2};
  for (int d = 0; d < 2; ++d) {
    /* S_{4+d} = m_0 (-K u + (ug - u)/theta) */
    J[4 + d][0] = -K * u[d] + (ug[d] - u[d]) * it;
    J[4 + d][2] = m0 * (K + it) * u[d] / m2;
    J[4 + d][4 + d] = -m0 * (K + it) / m2;
  }
  J[2][0] = -K;
  J[3][1] = -1.5 * K;
  if (K == 0.0) return;
  if (P->closure == 1) {
    /* The entropy maximiser's multipliers are fixed by the optimality
     * conditions F_k(lambda, m) = mu_{k+1}(lambda) - m_{k/2} = 0, whose
     * Jacobian in lambda is the Hessian H_kl = mu_{k+l+1} and in m is -I, so
     * d lambda / d m = H^{-1} (implicit function theorem). With
     * n(S=0) = exp(lambda_0) and m_{-1/2} = int S^{-1/2} n dS,
     *   d n0 / d lambda = (n0, 0, 0, 0),
     *   d m_{-1/2} / d lambda_l = int S^{-1/2} x^l n dS = mu_l,
     * so each row is H^{-1} applied to that gradient (H is symmetric). */
    double lam[4], mmh, n0, mu[8], H[4][4], g0[4], g1[4], a[4], b[4];
    if (orc_maxent(w, lam, &mmh, &n0)) {
      for (int l = 0; l < 4; ++l) J[0][l] = J[1][l] = NAN;
      return;
    }
    maxent_moments(lam, mu);
    for (int k = 0; k < 4; ++k) {
      for (int l = 0; l < 4; ++l) H[k][l] = mu[k + l + 1];
      g0[k] = k == 0 ? n0 : 0.0;
      g1[k] = mu[k];
    }
    if (spd_solve4(H, g0, a) || spd_solve4(H, g1, b)) {
      for (int l = 0; l < 4; ++l) J[0][l] = J[1][l] = NAN;
      return;
    }
    for (int l = 0; l < 4; ++l) {
      J[0][l] = -K * a[l];
      J[1][l] = -(K / 2.0) * b[l];
    }
    return;
  }
  double mmh, n0;
  lognormal_closure(P, w, &mmh, &n0);
  double L1 = log(m1 / m0), L2 = log(m2 / m0);
  double s2 = 4.0 * (L2 - 2.0 * L1);
  int clipped = s2 < 1e-8;
  if (clipped) s2 = 1e-8;
  double mu = 2.0 * L1 - s2 / 4.0;
  double z = log(P->s_eps) - mu;
  double dL1[3] = {-1.0 / m0, 1.0 / m1, 0.0};
  double dL2[3] = {-1.0 / m0, 0.0, 1.0 / m2};
  for (int l = 0; l < 3; ++l) {
    double ds2 = clipped ? 0.0 : 4.0 * (dL2[l] - 2.0 * dL1[l]);
    double dmu = 2.0 * dL1[l] - ds2 / 4.0;
    double dm0 = (l == 0) ? 1.0 / m0 : 0.0;
    double dlmmh = dm0 - dmu / 2.0 + ds2 / 8.0;
    double dln0 = dm0 - ds2 / (2.0 * s2) + z * dmu / s2 + z * z * ds2 / (2.0 * s2 * s2);
    J[1][l] = -(K / 2.0) * mmh * dlmmh;
    J[0][l] = -K * n0 * dln0;
  }
}

/* W* = W - [mux (F_E - F_W) + muy (G_N - G_S)] over the whole grid (the
 * transport half of the step, eq. VF_scheme with reading R1), neighbours
 * by the boundary rule. */
static void transport_star(const orc_params* P, const double* W, double dt,
                           double* Ws)
{
  int nv = orc_nvar(P->model), nx = P->nx, ny = P->ny;
  size_t plane = (size_t)nx * ny;
  double mux = dt / (P->lx / nx), muy = dt / (P->ly / ny);
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      double c[ORC_MAXV], nb[4][ORC_MAXV];
      int di[4] = {-1, 1, 0, 0}, dj[4] = {0, 0, -1, 1};
      for (int v = 0; v < nv; ++v) c[v] = W[v * plane + (size_t)j * nx + i];
      for (int s = 0; s < 4; ++s) {
        int ii = i + di[s], jj = j + dj[s];
        int out = ii < 0 || ii >= nx || jj < 0 || jj >= ny;
        if (P->bc == ORC_PERIODIC) {
          ii = (ii + nx) % nx;
          jj = (jj + ny) % ny;
        } else if (out && P->bc == ORC_TRANSMISSIVE) {
          ii = i;
          jj = j;
        }
        for (int v = 0; v < nv; ++v)
          nb[s][v] = (out && P->bc == ORC_DIRICHLET)
                         ? P->ghost[s][v]
                         : W[v * plane + (size_t)jj * nx + ii];
      }
      double FE[ORC_MAXV], FW[ORC_MAXV], GN[ORC_MAXV], GS[ORC_MAXV];
      num_flux(P, c, nb[ORC_EAST], 0, FE);
      num_flux(P, nb[ORC_WEST], c, 0, FW);
      num_flux(P, c, nb[ORC_NORTH], 1, GN);
      num_flux(P, nb[ORC_SOUTH], c, 1, GS);
      for (int v = 0; v < nv; ++v) {
        double t = mux * (FE[v] - FW[v]) + muy * (GN[v] - GS[v]);
        Ws[v * plane + (size_t)j * nx + i] = c[v] - t;
      }
    }
}

/* One adjoint step: lam_out = (dW^{n+1}/dW^n)^T lam_in at state W with time
 * step dt. For the spray, W^{n+1} = W* + dt S(W*) with W* the transport
 * step, so lam_in is first taken back through the source,
 * mu = lam_in + dt J_S(W*)^T lam_in, cell by cell, and then through the
 * transport. The transport part scatters over faces with explicit Jacobians.
 * A ghost cell has no update equation (its multiplier is zero); on a
 * transmissive boundary it is a copy of the boundary cell, so its
 * sensitivity goes to that cell; on a Dirichlet boundary it holds the
 * prescribed state, which does not depend on W, so its sensitivity is
 * dropped. ug: the spray's gas velocity (2 planes), unused otherwise. */
int orc_adjoint_step(const orc_params* P, const double* W, const double* ug,
                     double dt, const double* lam_in, double* lam_out)
{
  int rc = orc_validate(P);
  if (rc) return rc;
  int spray = P->model == ORC_SPRAY;
  if (spray && !ug) return ORC_EINVAL;
  int nv = orc_nvar(P->model), nx = P->nx, ny = P->ny;
  size_t plane = (size_t)nx * ny;
  int dir = P->bc == ORC_DIRICHLET;
  double mu[2] = {dt / (P->lx / nx), dt / (P->ly / ny)};
  int per = P->bc == ORC_PERIODIC;
  double* lam_src = NULL;
  const double* lm = lam_in; /* the multiplier of W* */
  if (spray) {
    double* Ws = (double*)malloc(sizeof(double) * nv * plane);
    lam_src = (double*)malloc(sizeof(double) * nv * plane);
    if (!Ws || !lam_src) { free(Ws); free(lam_src); return ORC_EINVAL; }
    transport_star(P, W, dt, Ws);
    for (size_t c = 0; c < plane; ++c) {
      double w[6], J[6][6], u2[2] = {ug[c], ug[plane + c]};
      for (int v = 0; v < 6; ++v) w[v] = Ws[v * plane + c];
      spray_source_jacobian(P, w, u2, J);
      for (int l = 0; l < 6; ++l) {
        double s = 0.0;
        for (int k = 0; k < 6; ++k) s = s + J[k][l] * lam_in[k * plane + c];
        lam_src[l * plane + c] = lam_in[l * plane + c] + dt * s;
      }
    }
    free(Ws);
    lm = lam_src;
  }
  memcpy(lam_out, lm, sizeof(double) * nv * plane);
  for (int d = 0; d < 2; ++d) {
    int n_along = d == 0 ? nx : ny, n_across = d == 0 ? ny : nx;
    int first = per ? 0 : -1;
    for (int a = 0; a < n_across; ++a)
      for (int f = first; f < n_along; ++f) {
        /* face between cell index f (left) and f+1 (right) along axis d */
        int il = f, ir = f + 1;
        int vl = 1, vr = 1; /* is the side a real cell with an update? */
        if (per) {
          ir = ir % n_along;
        } else {
          if (il < 0) { il = 0; vl = 0; }
          if (ir >= n_along) { ir = n_along - 1; vr = 0; }
        }
        size_t cl = d == 0 ? (size_t)a * nx + il : (size_t)il * nx + a;
        size_t cr = d == 0 ? (size_t)a * nx + ir : (size_t)ir * nx + a;
        double wl[ORC_MAXV], wr[ORC_MAXV], dl[ORC_MAXV];
        double JL[ORC_MAXV][ORC_MAXV], JR[ORC_MAXV][ORC_MAXV];
        for (int v = 0; v < nv; ++v) {
          wl[v] = W[v * plane + cl];
          wr[v] = W[v * plane + cr];
          /* Dirichlet ghosts: west/east along x, south/north along y */
          if (dir && !vl) wl[v] = P->ghost[d == 0 ? ORC_WEST : ORC_SOUTH][v];
          if (dir && !vr) wr[v] = P->ghost[d == 0 ? ORC_EAST : ORC_NORTH][v];
        }
        num_flux_jacobians(P, wl, wr, d, JL, JR);
        for (int v = 0; v < nv; ++v) {
          double lr = vr ? lm[v * plane + cr] : 0.0;
          double ll = vl ? lm[v * plane + cl] : 0.0;
          dl[v] = lr - ll;
        }
        for (int l = 0; l < nv; ++l) {
          double sL = 0.0, sR = 0.0;
          for (int k = 0; k < nv; ++k) {
            sL = sL + JL[k][l] * dl[k];
            sR = sR + JR[k][l] * dl[k];
          }
          if (vl || !dir) lam_out[l * plane + cl] = lam_out[l * plane + cl] + mu[d] * sL;
          if (vr || !dir) lam_out[l * plane + cr] = lam_out[l * plane + cr] + mu[d] * sR;
        }
      }
  }
  free(lam_src);
  return ORC_OK;
}

/* Gradient of a loss of the final state with respect to the initial state
 * for nsteps transport steps with the given dts (held fixed): the forward
 * states are all stored, then the adjoint steps run in reverse.
 * lam: in = dL/dW^N, out = dL/dW^0. */
int orc_adjoint_run(const orc_params* P, const double* W0, const double* ug,
                    int nsteps, const double* dts, double* lam)
{
  int rc = orc_validate(P);
  if (rc) return rc;
  if (P->model == ORC_SPRAY && !ug) return ORC_EINVAL;
  int nv = orc_nvar(P->model);
  size_t n = (size_t)nv * P->nx * P->ny;
  double* states = (double*)malloc(sizeof(double) * n * (nsteps > 0 ? nsteps : 1));
  double* tmp = (double*)malloc(sizeof(double) * n);
  if (!states || !tmp) { free(states); free(tmp); return ORC_EINVAL; }
  memcpy(states, W0, sizeof(double) * n);
  for (int k = 1; k < nsteps; ++k) {
    memcpy(states + (size_t)k * n, states + (size_t)(k - 1) * n, sizeof(double) * n);
    rc = orc_run_dts(P, states + (size_t)k * n, ug, 1, dts + (k - 1));
    if (rc) break;
  }
  for (int k = nsteps - 1; k >= 0 && rc == ORC_OK; --k) {
    rc = orc_adjoint_step(P, states + (size_t)k * n, ug, dts[k], lam, tmp);
    memcpy(lam, tmp, sizeof(double) * n);
  }
  free(states);
  free(tmp);
  return rc;
}
