// adjoint_emu.cpp -- runs the adjoint kernel's wave strips on the CPU, one
// host thread per lane in lockstep, to check memory bounds and to compare
// the two lane layouts without a GPU.
//
// Usage: adjoint_emu model bc nx ny ld layout rows [out]
//
// Buffers (W, lambda in, two lambda out) are exactly as large as the ABI
// contract (nVar * ny * ld doubles) and end where their allocation ends, so
// AddressSanitizer reports any access outside them. W is a smooth positive
// state, lambda a pseudo-random field. Both layouts run every tile; every
// grid cell must be written, no padding column touched, and the two
// results must agree bit for bit. With `out`, the file receives raw doubles:
// W and lambda (nVar * ny * nx each, compact), the one-cell layout's
// multipliers (the same shape), then the Dirichlet states (4 x nVar), for a
// comparison with the oracle's adjoint step (dt 1e-3, unit square).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <thread>
#include <vector>

thread_local emu_dim3 emu_threadIdx;
static std::barrier<>* g_bar;
static long long g_slot[64];
static thread_local int t_lane;

int emu_dpp(int x, int ctrl) {
  g_slot[t_lane] = x;
  g_bar->arrive_and_wait();
  const int src = ctrl == 0x130 ? t_lane + 1 : t_lane - 1;  // wave_shl:1 / wave_shr:1
  const int r = (src < 0 || src > 63) ? 0 : static_cast<int>(g_slot[src]);
  g_bar->arrive_and_wait();
  return r;
}

unsigned long long emu_shfl_xor(unsigned long long x, int o) {
  g_slot[t_lane] = static_cast<long long>(x);
  g_bar->arrive_and_wait();
  const unsigned long long r = static_cast<unsigned long long>(g_slot[t_lane ^ o]);
  g_bar->arrive_and_wait();
  return r;
}

#include "../../paper_1701_05431_amd/csrc/fvm_internal.hpp"
#include "../../paper_1701_05431_amd/csrc/fvm_models.hpp"
#include "../../paper_1701_05431_amd/csrc/fvm_adjoint.hpp"

using namespace fvm;

template <class M, int BC>
static void run_strip(const M& m, const AdjointArgs& a, int cpl, int xs, int j0, int j1,
                      double mux, double muy, bool down) {
  std::barrier<> bar(64);
  g_bar = &bar;
  std::vector<std::thread> lanes;
  for (int lane = 0; lane < 64; ++lane)
    lanes.emplace_back([&, lane] {
      t_lane = lane;
      emu_threadIdx = {static_cast<unsigned>(lane), 0, 0};
      if (xs >= a.g.nx) return;  // uniform: the whole wave leaves
      if (cpl == 1 && down)
        adjoint_strip1<M, BC, true>(m, a, xs, j0, j1, mux, muy);
      else if (cpl == 1)
        adjoint_strip1<M, BC, false>(m, a, xs, j0, j1, mux, muy);
      else if (xs + 2 * kWave <= a.g.nx)
        adjoint_strip2<M, BC, false>(m, a, xs, j0, j1, mux, muy);
      else
        adjoint_strip2<M, BC, true>(m, a, xs, j0, j1, mux, muy);
    });
  for (auto& t : lanes) t.join();
}

static double* exact_buffer(size_t n, double fill, std::vector<void*>& keep) {
  const size_t bytes = n * 8, padded = (bytes + 255) / 256 * 256;
  char* raw = static_cast<char*>(aligned_alloc(256, padded));
  keep.push_back(raw);
  double* p = reinterpret_cast<double*>(raw + (padded - bytes));
  for (size_t k = 0; k < n; ++k) p[k] = fill;
  return p;
}

int main(int argc, char** argv) {
  if (argc != 8 && argc != 9) {
    std::fprintf(stderr, "usage: %s model bc nx ny ld layout rows [out]\n", argv[0]);
    return 2;
  }
  const int model = atoi(argv[1]), bc = atoi(argv[2]), nx = atoi(argv[3]), ny = atoi(argv[4]);
  const int ld = atoi(argv[5]), layout = atoi(argv[6]), rows = atoi(argv[7]);
  const int nv = model == 0 ? 1 : 4;
  if (ld % 2) {
    std::fprintf(stderr, "two cells per lane needs an even pitch\n");
    return 2;
  }
  GridGeom g{};
  g.nx = nx;
  g.ny = ny;
  g.bc = bc;
  if (layout == 1) {
    g.ld = nv * ld;
    g.plane = ld;
  } else {
    g.ld = ld;
    g.plane = static_cast<size_t>(ld) * ny;
  }
  g.dx = 1.0 / nx;
  g.dy = 1.0 / ny;
  std::vector<void*> keep;
  const size_t elems = static_cast<size_t>(nv) * ny * ld;
  double* w = exact_buffer(elems, 1.0, keep);
  double* lin = exact_buffer(elems, 0.0, keep);
  double* out1 = exact_buffer(elems, __builtin_nan(""), keep);
  double* out2 = exact_buffer(elems, __builtin_nan(""), keep);
  auto at = [&](double* b, int v, int j, int i) -> double& {
    return b[v * g.plane + static_cast<size_t>(j) * g.ld + i];
  };
  unsigned long long seed = 12345;
  auto rnd = [&] {
    seed = seed * 6364136223846793005ull + 1442695040888963407ull;
    return static_cast<double>(seed >> 11) / 9007199254740992.0 - 0.5;
  };
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const double x = (i + 0.5) / nx, y = (j + 0.5) / ny;
      if (nv == 4) {
        const double r = 1.0 + 0.3 * std::sin(6.0 * x) * std::cos(5.0 * y);
        const double u = 0.4 * std::cos(3.0 * y), v = -0.3 * std::sin(4.0 * x);
        const double p = 1.0 + 0.2 * std::cos(7.0 * x + 2.0 * y);
        at(w, 0, j, i) = r;
        at(w, 1, j, i) = r * u;
        at(w, 2, j, i) = r * v;
        at(w, 3, j, i) = p / 0.4 + 0.5 * r * (u * u + v * v);
      } else {
        at(w, 0, j, i) = std::sin(6.0 * x + 3.0 * y);
      }
      for (int vv = 0; vv < nv; ++vv) at(lin, vv, j, i) = rnd();
    }
  // Dirichlet (bc 2): ghost states a little off the interior values
  double ghost[4 * kMaxVar] = {};
  for (int side = 0; side < 4; ++side)
    for (int v = 0; v < nv; ++v) ghost[side * kMaxVar + v] = (1.05 + 0.1 * side) * at(w, v, 0, 0);
  ModelConsts mc{};
  mc.gamma = 1.4;
  mc.gm1 = 0.4;
  mc.ax = 0.7;
  mc.ay = -0.4;
  const double dt = 1e-3, mux = dt / g.dx, muy = dt / g.dy;
  for (int cpl = 1; cpl <= 2; ++cpl) {
    AdjointArgs a{};
    a.w = w;
    a.lam_in = lin;
    a.lam_out = cpl == 1 ? out1 : out2;
    a.dt_arg = dt;
    a.g = g;
    for (int k = 0; k < 4 * kMaxVar; ++k) a.ghost[k] = ghost[k];
    const int sw = cpl == 1 ? kOutPerWave : 2 * kWave;
    const int nstrip = (nx + sw - 1) / sw, tiles_y = (ny + rows - 1) / rows;
    for (int ty = 0; ty < tiles_y; ++ty)
      for (int sx = 0; sx < nstrip; ++sx) {
        const int xs = sx * sw, j0 = ty * rows, j1 = std::min(j0 + rows, ny);
        auto go = [&](auto bct) {
          constexpr int B = decltype(bct)::value;
          // the one-cell strips of odd tile rows march down, as in the kernel
          const bool down = (ty & 1) != 0;
          if (model == 0)
            run_strip<AdjAdv, B>(AdjAdv(mc), a, cpl, xs, j0, j1, mux, muy, down);
          else
            run_strip<AdjEuler, B>(AdjEuler(mc), a, cpl, xs, j0, j1, mux, muy, down);
        };
        if (bc == 0) go(std::integral_constant<int, 0>());
        else if (bc == 1) go(std::integral_constant<int, 1>());
        else go(std::integral_constant<int, 2>());
      }
  }
  long missing = 0, stray = 0, differ = 0;
  for (int v = 0; v < nv; ++v)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < ld; ++i) {
        const double o1 = at(out1, v, j, i), o2 = at(out2, v, j, i);
        if (i >= nx) {
          stray += !std::isnan(o1) + !std::isnan(o2);
        } else {
          missing += std::isnan(o1) + std::isnan(o2);
          differ += std::memcmp(&o1, &o2, 8) != 0;
        }
      }
  if (argc == 9) {
    std::vector<double> dump;
    for (double* b : {w, lin, out1})
      for (int v = 0; v < nv; ++v)
        for (int j = 0; j < ny; ++j)
          for (int i = 0; i < nx; ++i) dump.push_back(at(b, v, j, i));
    for (int side = 0; side < 4; ++side)
      for (int v = 0; v < nv; ++v) dump.push_back(ghost[side * kMaxVar + v]);
    std::FILE* f = std::fopen(argv[8], "wb");
    if (!f || std::fwrite(dump.data(), 8, dump.size(), f) != dump.size()) return 3;
    std::fclose(f);
  }
  std::printf("model=%d bc=%d %dx%d ld=%d layout=%d rows=%d missing=%ld stray=%ld differ=%ld\n",
              model, bc, nx, ny, ld, layout, rows, missing, stray, differ);
  for (void* p : keep) free(p);
  return (missing || stray || differ) ? 1 : 0;
}
