// fvm_adjoint_spray.hip -- launch of the spray adjoint (the device code and
// its derivation are in fvm_adjoint_spray.hpp): one thread per cell, rows of
// 64 cells per wave, four rows per workgroup.
#include <hip/hip_runtime.h>

#include "fvm_adjoint_spray.hpp"
#include "fvm_internal.hpp"

namespace fvm {

namespace {

constexpr int kSaThreads = 256;
constexpr int kSaX = 64;  // cells of one row per wave
constexpr int kSaY = kSaThreads / kSaX;

__global__ __launch_bounds__(kSaThreads) void spray_adjoint_kernel(AdjointArgs a,
                                                                  const double* ug,
                                                                  int tiles_x) {
  const int b = static_cast<int>(blockIdx.x);
  const int i = (b % tiles_x) * kSaX + static_cast<int>(threadIdx.x) % kSaX;
  const int j = (b / tiles_x) * kSaY + static_cast<int>(threadIdx.x) / kSaX;
  if (i >= a.g.nx || j >= a.g.ny) return;
  sadj::spray_adjoint_cell(a, ug, j, i);
}

}  // namespace

hipError_t launch_spray_adjoint(const AdjointArgs& a, const double* ug, hipStream_t st) {
  if (!a.w || !a.lam_in || !a.lam_out || !ug || a.g.nx < 1 || a.g.ny < 1)
    return hipErrorInvalidValue;
  const long long tx = (a.g.nx + kSaX - 1) / kSaX;
  const long long ty = (a.g.ny + kSaY - 1) / kSaY;
  if (tx * ty > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(spray_adjoint_kernel, dim3(static_cast<unsigned>(tx * ty)),
                     dim3(kSaThreads), 0, st, a, ug, static_cast<int>(tx));
  return hipGetLastError();
}

}  // namespace fvm
