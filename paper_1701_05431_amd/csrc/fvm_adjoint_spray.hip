// fvm_adjoint_spray.hip -- launch of the spray adjoint (the device code and
// its derivation are in fvm_adjoint_spray.hpp): one workgroup per tile of
// 64 x 16 cells (512 threads), mu of the tile and its ring in LDS, one
// barrier. Measured on the 2048^2 spray: 64 x 16 with 512 threads 261 us per
// step, 64 x 8 with 256 threads 278, 64 x 4 318, 64 x 32 288.
#include <hip/hip_runtime.h>

#include "fvm_adjoint_spray.hpp"
#include "fvm_internal.hpp"
#include "fvm_step.hpp"

namespace fvm {

namespace {

__global__ __launch_bounds__(sadj::kTileThreads) void spray_adjoint_kernel(AdjointArgs a,
                                                                          const double* ug,
                                                                          int tiles_x,
                                                                          int ntiles) {
  __shared__ double mu_s[6 * sadj::kRing];
  // each XCD takes a contiguous row-major range of tiles, so the halo
  // columns and rows a tile shares with its neighbours stay in that XCD's L2
  const int b = xcd_tile(static_cast<int>(blockIdx.x), ntiles);
  const int i0 = (b % tiles_x) * sadj::kTX, j0 = (b / tiles_x) * sadj::kTY;
  const sadj::SprayAdj s = sadj::make_adj(a, ug);
  const int tid = static_cast<int>(threadIdx.x);
  sadj::tile_mu(s, j0, i0, tid, mu_s);
  __syncthreads();
  sadj::tile_out(s, j0, i0, tid, mu_s);
}

}  // namespace

hipError_t launch_spray_adjoint(const AdjointArgs& a, const double* ug, hipStream_t st) {
  if (!a.w || !a.lam_in || !a.lam_out || !ug || a.g.nx < 1 || a.g.ny < 1)
    return hipErrorInvalidValue;
  const long long tx = (a.g.nx + sadj::kTX - 1) / sadj::kTX;
  const long long ty = (a.g.ny + sadj::kTY - 1) / sadj::kTY;
  if (tx * ty > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(spray_adjoint_kernel, dim3(static_cast<unsigned>(tx * ty)),
                     dim3(sadj::kTileThreads), 0, st, a, ug, static_cast<int>(tx),
                     static_cast<int>(tx * ty));
  return hipGetLastError();
}

}  // namespace fvm
