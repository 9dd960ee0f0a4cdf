// strip_emu.cpp -- runs the device code of the fused step's wave strips on
// the CPU, one host thread per lane, to check memory bounds and coverage
// without a GPU.
//
// Build: clang++ -std=c++20 -fsanitize=address -I tests/emu/shim ...
// Usage: strip_emu model bc nx ny ld layout cells_per_lane rows waves_per_block
//
// Every buffer is exactly as large as the library's contract says (state:
// nVar * ny * ld doubles; spray gas velocity: 2 * ny * ld) and ends where the
// allocation ends, so AddressSanitizer reports any access outside it. The
// output starts as NaN; after every tile of the grid has run, each cell of
// the grid must have been written and each padding column (i >= nx) must not.
// The input is a uniform state, which the step leaves bitwise unchanged
// (advection and Euler: equal fluxes cancel; spray: K = 0 and the gas velocity
// equals the droplet velocity, so the source vanishes); Dirichlet ghosts
// (bc 2) hold the same state.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <thread>
#include <type_traits>
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
#include "../../paper_1701_05431_amd/csrc/fvm_step.hpp"

using namespace fvm;

// One wave strip, dispatched as the step kernel does.
template <class M, int BC>
static void run_strip(const M& m, const double* win, double* wout, const double* ug,
                      const GridGeom& g, int cpl, int xs, int j0, int j1, double mux, double muy,
                      double dt, const double* gh, bool down) {
  std::barrier<> bar(64);
  g_bar = &bar;
  std::vector<std::thread> lanes;
  for (int lane = 0; lane < 64; ++lane)
    lanes.emplace_back([&, lane] {
      t_lane = lane;
      emu_threadIdx = {static_cast<unsigned>(lane), 0, 0};
      unsigned long long bx = 0, by = 0;
      if (xs >= g.nx) return;  // uniform: the whole wave leaves
      if (cpl == 1) {
        if (xs + kWave <= g.nx)
          march_strip1<M, BC, false>(m, win, wout, ug, g, xs, j0, j1, mux, muy, dt, bx, by, gh);
        else
          march_strip1<M, BC, true>(m, win, wout, ug, g, xs, j0, j1, mux, muy, dt, bx, by, gh);
      } else {
        constexpr int PF = M::kPrefetch2;
        if (xs + 2 * kWave <= g.nx && down)
          march_strip2<M, BC, false, PF, false, true>(m, win, wout, ug, g, xs, j0, j1, mux, muy,
                                                      dt, bx, by, gh);
        else if (xs + 2 * kWave <= g.nx)
          march_strip2<M, BC, false>(m, win, wout, ug, g, xs, j0, j1, mux, muy, dt, bx, by, gh);
        else if (down)
          march_strip2<M, BC, true, PF, false, true>(m, win, wout, ug, g, xs, j0, j1, mux, muy,
                                                     dt, bx, by, gh);
        else
          march_strip2<M, BC, true>(m, win, wout, ug, g, xs, j0, j1, mux, muy, dt, bx, by, gh);
      }
    });
  for (auto& t : lanes) t.join();
}

// A buffer of n doubles whose last element is the last byte of its
// allocation; the start keeps 16-byte alignment when n is even.
static double* exact_buffer(size_t n, double fill, std::vector<void*>& keep) {
  const size_t bytes = n * 8, padded = (bytes + 255) / 256 * 256;
  char* raw = static_cast<char*>(aligned_alloc(256, padded));
  keep.push_back(raw);
  // aligned_alloc hands out `padded` bytes; the checked region is its tail
  double* p = reinterpret_cast<double*>(raw + (padded - bytes));
  for (size_t k = 0; k < n; ++k) p[k] = fill;
  return p;
}

int main(int argc, char** argv) {
  if (argc != 10) {
    std::fprintf(stderr, "usage: %s model bc nx ny ld layout cpl rows wpb\n", argv[0]);
    return 2;
  }
  const int model = atoi(argv[1]), bc = atoi(argv[2]), nx = atoi(argv[3]), ny = atoi(argv[4]);
  const int ld = atoi(argv[5]), layout = atoi(argv[6]), cpl = atoi(argv[7]);
  const int rows = atoi(argv[8]), wpb = atoi(argv[9]);
  // model 3: the spray's transport-only strip (entropy-maximising closure),
  // which must not touch the gas velocity: it gets none
  const int nv = model == 0 ? 1 : (model == 1 ? 4 : 6);
  if (cpl == 2 && ((ld % 2) || (static_cast<size_t>(nv) * ny * ld) % 2)) {
    std::fprintf(stderr, "two cells per lane needs an even pitch\n");
    return 2;
  }
  // the library's geometry of the two layouts
  GridGeom g{};
  g.nx = nx;
  g.ny = ny;
  g.bc = bc;
  if (layout == 1) {
    g.ld = nv * ld;
    g.plane = ld;
    g.uld = 2 * ld;
    g.uplane = ld;
  } else {
    g.ld = ld;
    g.plane = static_cast<size_t>(ld) * ny;
    g.uld = ld;
    g.uplane = g.plane;
  }
  g.dx = 1.0 / nx;
  g.dy = 1.0 / ny;
  g.cfl = 0.45;
  g.hmin = g.dx < g.dy ? g.dx : g.dy;

  std::vector<void*> keep;
  const size_t elems = static_cast<size_t>(nv) * ny * ld;
  double* win = exact_buffer(elems, 1.0, keep);
  double* wout = exact_buffer(elems, __builtin_nan(""), keep);
  double* ug = nullptr;
  auto at = [&](double* w, int v, int j, int i) -> double& {
    return w[v * g.plane + static_cast<size_t>(j) * g.ld + i];
  };
  if (model == 1)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        at(win, 1, j, i) = 0.25;
        at(win, 2, j, i) = -0.125;
        at(win, 3, j, i) = 2.5;
      }
  if (model >= 2) {
    // moments of one size distribution, velocity 0.5 in x; gas alike
    if (model == 2) ug = exact_buffer(2ull * ny * ld, 0.0, keep);
    const double m[4] = {1.0, 0.45, 0.25, 0.15};
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        for (int v = 0; v < 4; ++v) at(win, v, j, i) = m[v];
        at(win, 4, j, i) = 0.5 * m[2];
        at(win, 5, j, i) = 0.0;
        if (ug) ug[static_cast<size_t>(j) * g.uld + i] = 0.5;
      }
  }
  ModelConsts mc{};
  mc.gamma = 1.4;
  mc.gm1 = 0.4;
  mc.ax = 1.0;
  mc.ay = -0.5;
  mc.K = 0.0;
  mc.inv_theta = 10.0;
  mc.s_eps = 0.01;
  mc.log_s_eps = std::log(0.01);

  // Dirichlet ghosts: the uniform state on every side
  double gh[4 * kMaxVar] = {};
  for (int side = 0; side < 4; ++side)
    for (int v = 0; v < nv; ++v) gh[side * kMaxVar + v] = at(win, v, 0, 0);

  // the step kernel's tiles: WPB strips side by side, `rows` rows each
  const int sw = strip_width(cpl);
  const int tiles_x = (nx + sw * wpb - 1) / (sw * wpb), tiles_y = (ny + rows - 1) / rows;
  const double dt = 1e-3, mux = dt / g.dx, muy = dt / g.dy;
  for (int ty = 0; ty < tiles_y; ++ty)
    for (int tx = 0; tx < tiles_x; ++tx)
      for (int w = 0; w < wpb; ++w) {
        const int xs = (tx * wpb + w) * sw, j0 = ty * rows, j1 = std::min(j0 + rows, ny);
        // two-cells-per-lane strips of odd tile rows march down, as in the kernel
        const bool down = (ty & 1) != 0;
        auto go = [&](auto bct) {
          constexpr int B = decltype(bct)::value;
          if (model == 0)
            run_strip<Adv, B>(Adv(mc), win, wout, ug, g, cpl, xs, j0, j1, mux, muy, dt, gh, down);
          else if (model == 1)
            run_strip<Euler, B>(Euler(mc), win, wout, ug, g, cpl, xs, j0, j1, mux, muy, dt, gh,
                                down);
          else if (model == 2)
            run_strip<Spray, B>(Spray(mc), win, wout, ug, g, cpl, xs, j0, j1, mux, muy, dt, gh,
                                down);
          else
            run_strip<SprayTransport, B>(SprayTransport(mc), win, wout, ug, g, cpl, xs, j0, j1,
                                         mux, muy, dt, gh, down);
        };
        if (bc == 0) go(std::integral_constant<int, 0>());
        else if (bc == 1) go(std::integral_constant<int, 1>());
        else go(std::integral_constant<int, 2>());
      }

  long missing = 0, stray = 0, changed = 0;
  for (int v = 0; v < nv; ++v)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < ld; ++i) {
        const double o = at(wout, v, j, i);
        if (i >= nx) {
          stray += !std::isnan(o);
        } else if (std::isnan(o)) {
          ++missing;
        } else {
          changed += o != at(win, v, j, i);
        }
      }
  std::printf("model=%d bc=%d %dx%d ld=%d layout=%d cpl=%d rows=%d wpb=%d missing=%ld stray=%ld "
              "changed=%ld\n", model, bc, nx, ny, ld, layout, cpl, rows, wpb, missing, stray,
              changed);
  for (void* p : keep) free(p);
  return (missing || stray || changed) ? 1 : 0;
}
