// spray_adjoint_emu.cpp -- runs the spray adjoint's device code on the CPU,
// tile by tile and thread by thread, to check its memory accesses (global
// and LDS) and its values without a GPU.
//
// Usage: spray_adjoint_emu bc nx ny pitch layout lx ly dt K inv_theta s_eps in out
//
// `in` holds, as raw doubles: W and lambda (6 * ny * nx each, planar, no
// padding), u_g (2 * ny * nx) and the Dirichlet states (4 sides x 6). They are
// copied into buffers laid out as the library lays them out (pitch, layout)
// and exactly as large as the ABI contract, so AddressSanitizer reports any
// access outside them; the padding columns of the output start as NaN and
// must stay untouched. `out` receives lambda^n (6 * ny * nx, planar).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

thread_local emu_dim3 emu_threadIdx;
int emu_dpp(int x, int) { return x; }
unsigned long long emu_shfl_xor(unsigned long long x, int) { return x; }

#include "../../paper_1701_05431_amd/csrc/fvm_internal.hpp"
#include "../../paper_1701_05431_amd/csrc/fvm_adjoint_spray.hpp"

using namespace fvm;

int main(int argc, char** argv) {
  if (argc != 14) {
    std::fprintf(stderr, "usage: bc nx ny pitch layout lx ly dt K inv_theta s_eps in out\n");
    return 2;
  }
  const int bc = std::atoi(argv[1]), nx = std::atoi(argv[2]), ny = std::atoi(argv[3]);
  const int pitch = std::atoi(argv[4]), layout = std::atoi(argv[5]);
  const double lx = std::atof(argv[6]), ly = std::atof(argv[7]), dt = std::atof(argv[8]);
  const double K = std::atof(argv[9]), inv_theta = std::atof(argv[10]);
  const double s_eps = std::atof(argv[11]);
  if (nx < 1 || ny < 1 || pitch < nx) return 2;
  const size_t n = static_cast<size_t>(nx) * ny;
  std::vector<double> raw(6 * n * 2 + 2 * n + 24);
  std::FILE* f = std::fopen(argv[12], "rb");
  if (!f || std::fread(raw.data(), sizeof(double), raw.size(), f) != raw.size()) return 3;
  std::fclose(f);

  GridGeom g{};
  g.nx = nx;
  g.ny = ny;
  g.bc = bc;
  if (layout == 1) {
    g.ld = 6 * pitch;
    g.plane = static_cast<size_t>(pitch);
    g.uld = 2 * pitch;
    g.uplane = static_cast<size_t>(pitch);
  } else {
    g.ld = pitch;
    g.plane = static_cast<size_t>(pitch) * ny;
    g.uld = pitch;
    g.uplane = g.plane;
  }
  g.dx = lx / nx;
  g.dy = ly / ny;
  const size_t total = static_cast<size_t>(pitch) * ny * 6;  // nVar * ny * pitch
  const size_t utotal = static_cast<size_t>(pitch) * ny * 2;
  // exactly sized heap buffers
  double* w = new double[total];
  double* li = new double[total];
  double* lo = new double[total];
  double* ug = new double[utotal];
  for (size_t k = 0; k < total; ++k) w[k] = li[k] = lo[k] = NAN;
  for (size_t k = 0; k < utotal; ++k) ug[k] = NAN;
  for (int v = 0; v < 6; ++v)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        const size_t at = v * g.plane + static_cast<size_t>(j) * g.ld + i;
        w[at] = raw[v * n + static_cast<size_t>(j) * nx + i];
        li[at] = raw[6 * n + v * n + static_cast<size_t>(j) * nx + i];
      }
  for (int v = 0; v < 2; ++v)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i)
        ug[v * g.uplane + static_cast<size_t>(j) * g.uld + i] =
            raw[12 * n + v * n + static_cast<size_t>(j) * nx + i];

  AdjointArgs a{};
  a.w = w;
  a.lam_in = li;
  a.lam_out = lo;
  a.dts = nullptr;
  a.dt_arg = dt;
  a.g = g;
  a.m.K = K;
  a.m.inv_theta = inv_theta;
  a.m.s_eps = s_eps;
  a.m.log_s_eps = std::log(s_eps);
  for (int s = 0; s < 4; ++s)
    for (int v = 0; v < 6; ++v) a.ghost[s * kMaxVar + v] = raw[14 * n + s * 6 + v];

  // every tile's three phases, thread by thread, with a heap LDS stand-in of
  // exactly the kernel's size (the barriers sit between the phases)
  const sadj::SprayAdj sa = sadj::make_adj(a, ug);
  const int tx = (nx + sadj::kTX - 1) / sadj::kTX, ty = (ny + sadj::kTY - 1) / sadj::kTY;
  for (int b = 0; b < tx * ty; ++b) {
    const int i0 = (b % tx) * sadj::kTX, j0 = (b / tx) * sadj::kTY;
    double* lds = new double[sadj::kLdsDoubles];
    for (int k = 0; k < sadj::kLdsDoubles; ++k) lds[k] = NAN;
    double* box = lds;
    double* mu_s = lds + sadj::kBoxVars * sadj::kBox;
    // each thread's prefetched values (registers on the GPU)
    std::vector<double> pre(static_cast<size_t>(sadj::kTileThreads) * sadj::kMuPasses * sadj::kPre);
    for (int t = 0; t < sadj::kTileThreads; ++t) {
      double* q = pre.data() + static_cast<size_t>(t) * sadj::kMuPasses * sadj::kPre;
      sadj::tile_prefetch(sa, j0, i0, t, q);
      sadj::tile_load(sa, j0, i0, t, box);
    }
    for (int t = 0; t < sadj::kTileThreads; ++t)
      sadj::tile_mu(sa, j0, i0, t, box,
                    pre.data() + static_cast<size_t>(t) * sadj::kMuPasses * sadj::kPre, mu_s);
    for (int t = 0; t < sadj::kTileThreads; ++t) sadj::tile_out(sa, j0, i0, t, box, mu_s);
    delete[] lds;
  }

  // every cell written, no padding touched
  std::vector<double> res(6 * n);
  for (int v = 0; v < 6; ++v)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < pitch; ++i) {
        const double x = lo[v * g.plane + static_cast<size_t>(j) * g.ld + i];
        if (i < nx) {
          res[v * n + static_cast<size_t>(j) * nx + i] = x;
        } else if (!std::isnan(x)) {
          std::fprintf(stderr, "padding written at v=%d j=%d i=%d\n", v, j, i);
          return 4;
        }
      }
  f = std::fopen(argv[13], "wb");
  if (!f || std::fwrite(res.data(), sizeof(double), res.size(), f) != res.size()) return 3;
  std::fclose(f);
  delete[] w;
  delete[] li;
  delete[] lo;
  delete[] ug;
  std::puts("ok");
  return 0;
}
