// resident_emu.cpp -- runs the device code of the resident run (a whole
// adaptive run of a small grid in one workgroup) on the CPU: every cell's
// update from the LDS state (an exactly sized heap array here), then the
// maxima and the next dt, step after step, as the kernel's threads and its
// thread 0 do. AddressSanitizer reports any access outside the state arrays,
// the gas velocity or the ghost states.
//
// Usage: resident_emu model bc nx ny nsteps cfl in out
//   model 0 advection (a = (1, 0.5)), 1 Euler (gamma 1.4), 2 spray
//   (K = 1, theta = 0.1, S_eps = 0.01); unit square.
// `in` holds raw doubles: W (nVar * ny * nx, planar), then for the spray u_g
// (2 * ny * nx), then the Dirichlet states (4 sides x nVar). `out` receives
// W^n (nVar * ny * nx) followed by the n dts.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

thread_local emu_dim3 emu_threadIdx;
int emu_dpp(int x, int) { return x; }
unsigned long long emu_shfl_xor(unsigned long long x, int) { return x; }

#include "../../paper_1701_05431_amd/csrc/fvm_internal.hpp"
#include "../../paper_1701_05431_amd/csrc/fvm_resident.hpp"

using namespace fvm;

template <class M, int BC>
static void run(const StepArgs& a, double* A, double* B, int ncell, int nsteps, double dt0,
                std::vector<double>& dts) {
  const M m(a.m);
  double dt = dt0;
  for (int k = 0; k < nsteps; ++k) {
    const double mux = dt / a.g.dx, muy = dt / a.g.dy;
    unsigned long long bx = 0, by = 0;
    for (int c = 0; c < ncell; ++c) {
      const res::Cell r = res::cell_at<BC>(a.g, c);
      const double ugx = a.ug ? a.ug[r.uc] : 0.0, ugy = a.ug ? a.ug[a.g.uplane + r.uc] : 0.0;
      res::update_cell<M>(m, a.ghost, A, B, ncell, r, ugx, ugy, mux, muy, dt, bx, by);
    }
    unsigned int st = 0;
    const double dtn = res::next_step_dt(a.g, __longlong_as_double(static_cast<long long>(bx)),
                                         __longlong_as_double(static_cast<long long>(by)), st);
    dts.push_back(dt);
    dt = dtn;
    double* t = A;
    A = B;
    B = t;
  }
  if (nsteps % 2)  // the final state into the first array
    for (int q = 0; q < M::NV * ncell; ++q) B[q] = A[q];
}

template <class M>
static void run_bc(int bc, const StepArgs& a, double* A, double* B, int ncell, int nsteps,
                   double dt0, std::vector<double>& dts) {
  if (bc == 0) run<M, 0>(a, A, B, ncell, nsteps, dt0, dts);
  else if (bc == 1) run<M, 1>(a, A, B, ncell, nsteps, dt0, dts);
  else run<M, 2>(a, A, B, ncell, nsteps, dt0, dts);
}

int main(int argc, char** argv) {
  if (argc != 9) {
    std::fprintf(stderr, "usage: model bc nx ny nsteps cfl in out\n");
    return 2;
  }
  const int model = std::atoi(argv[1]), bc = std::atoi(argv[2]);
  const int nx = std::atoi(argv[3]), ny = std::atoi(argv[4]), nsteps = std::atoi(argv[5]);
  const double cfl = std::atof(argv[6]);
  if (model < 0 || model > 2 || bc < 0 || bc > 2 || nx < 1 || ny < 1 || nsteps < 0) return 2;
  const int nv = model == 0 ? 1 : (model == 1 ? 4 : 6);
  const int ncell = nx * ny;
  if (2LL * nv * ncell > kResidentDoubles) return 2;
  const size_t nin = static_cast<size_t>(nv) * ncell + (model == 2 ? 2 * ncell : 0) + 4 * nv;
  std::vector<double> raw(nin);
  std::FILE* f = std::fopen(argv[7], "rb");
  if (!f || std::fread(raw.data(), sizeof(double), raw.size(), f) != raw.size()) return 3;
  std::fclose(f);

  StepArgs a{};
  a.g.nx = nx;
  a.g.ny = ny;
  a.g.bc = bc;
  a.g.dx = 1.0 / nx;
  a.g.dy = 1.0 / ny;
  a.g.cfl = cfl;
  a.g.dt_max = 0.0;
  a.g.ld = nx;
  a.g.plane = static_cast<size_t>(ncell);
  a.g.uld = nx;
  a.g.uplane = static_cast<size_t>(ncell);
  a.m.ax = 1.0;
  a.m.ay = 0.5;
  a.m.gamma = 1.4;
  a.m.gm1 = 0.4;
  a.m.K = 1.0;
  a.m.inv_theta = 10.0;
  a.m.s_eps = 0.01;
  a.m.log_s_eps = std::log(0.01);
  // exactly sized arrays: the two LDS states, the gas velocity
  double* A = new double[static_cast<size_t>(nv) * ncell];
  double* B = new double[static_cast<size_t>(nv) * ncell];
  for (int q = 0; q < nv * ncell; ++q) {
    A[q] = raw[q];
    B[q] = NAN;
  }
  double* ug = nullptr;
  if (model == 2) {
    ug = new double[2 * static_cast<size_t>(ncell)];
    for (int q = 0; q < 2 * ncell; ++q) ug[q] = raw[static_cast<size_t>(nv) * ncell + q];
  }
  a.ug = ug;
  const double* gh = raw.data() + nin - 4 * nv;
  for (int s = 0; s < 4; ++s)
    for (int v = 0; v < nv; ++v) a.ghost[s * kMaxVar + v] = gh[s * nv + v];

  // the first dt: the speeds of the initial state, as the CFL launch
  unsigned long long bx = 0, by = 0;
  auto first = [&](auto m) {
    for (int c = 0; c < ncell; ++c) {
      double w[6], sx, sy;
      for (int v = 0; v < nv; ++v) w[v] = A[v * ncell + c];
      m.speeds(w, sx, sy);
      bx = umax64(bx, bits(sx));
      by = umax64(by, bits(sy));
    }
  };
  if (model == 0) first(Adv(a.m));
  else if (model == 1) first(Euler(a.m));
  else first(Spray(a.m));
  unsigned int st = 0;
  const double dt0 = res::next_step_dt(a.g, __longlong_as_double(static_cast<long long>(bx)),
                                       __longlong_as_double(static_cast<long long>(by)), st);
  std::vector<double> dts;
  if (model == 0) run_bc<Adv>(bc, a, A, B, ncell, nsteps, dt0, dts);
  else if (model == 1) run_bc<Euler>(bc, a, A, B, ncell, nsteps, dt0, dts);
  else run_bc<Spray>(bc, a, A, B, ncell, nsteps, dt0, dts);

  std::vector<double> out(A, A + static_cast<size_t>(nv) * ncell);
  out.insert(out.end(), dts.begin(), dts.end());
  f = std::fopen(argv[8], "wb");
  if (!f || std::fwrite(out.data(), sizeof(double), out.size(), f) != out.size()) return 3;
  std::fclose(f);
  delete[] A;
  delete[] B;
  delete[] ug;
  return 0;
}
