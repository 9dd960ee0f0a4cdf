// fvm_adjoint_spray.hip -- launch of the spray adjoint (the device code and
// its derivation are in fvm_adjoint_spray.hpp): one workgroup per tile of
// kTX x kTY cells; the tile's states with a two-cell ring, then mu of the
// tile with a one-cell ring, in LDS, two barriers.
#include <hip/hip_runtime.h>

#include "fvm_adjoint_spray.hpp"
#include "fvm_internal.hpp"
#include "fvm_step.hpp"

namespace fvm {

namespace {

template <bool SRC>
__global__ __launch_bounds__(sadj::kTileThreads) void spray_adjoint_kernel(AdjointArgs a,
                                                                          const double* ug,
                                                                          int tiles_x,
                                                                          int ntiles) {
  __shared__ double lds[sadj::kLdsDoubles];
  double* const box = lds;
  double* const mu_s = lds + sadj::kBoxVars * sadj::kBox;
  // each XCD takes a contiguous row-major range of tiles, so the ring rows
  // and columns a tile shares with its neighbours stay in that XCD's L2
  const int b = xcd_tile(static_cast<int>(blockIdx.x), ntiles);
  const int i0 = (b % tiles_x) * sadj::kTX, j0 = (b / tiles_x) * sadj::kTY;
  const sadj::SprayAdj s = sadj::make_adj(a, ug);
  const int tid = static_cast<int>(threadIdx.x);
  double pre[sadj::kMuPasses * sadj::kPre];
  sadj::tile_prefetch(s, j0, i0, tid, pre);
  sadj::tile_load(s, j0, i0, tid, box);
  __syncthreads();
  sadj::tile_mu<SRC>(s, j0, i0, tid, box, pre, mu_s);
  __syncthreads();
  sadj::tile_out(s, j0, i0, tid, box, mu_s);
}

}  // namespace

// src: the whole step's adjoint (source, then transport); otherwise the
// transport's alone, lam_in holding mu (the entropy closure's step, whose
// source adjoint runs first in its own pass).
hipError_t launch_spray_adjoint(const AdjointArgs& a, const double* ug, hipStream_t st,
                                bool src) {
  if (!a.w || !a.lam_in || !a.lam_out || !ug || a.g.nx < 1 || a.g.ny < 1)
    return hipErrorInvalidValue;
  const long long tx = (a.g.nx + sadj::kTX - 1) / sadj::kTX;
  const long long ty = (a.g.ny + sadj::kTY - 1) / sadj::kTY;
  if (tx * ty > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(src ? spray_adjoint_kernel<true> : spray_adjoint_kernel<false>,
                     dim3(static_cast<unsigned>(tx * ty)),
                     dim3(sadj::kTileThreads), 0, st, a, ug, static_cast<int>(tx),
                     static_cast<int>(tx * ty));
  return hipGetLastError();
}

}  // namespace fvm
