// logd_emu.cpp -- the kernels' logarithm (fvm_models.hpp, logd) built for
// the host: prints, for each argument read from stdin, the argument and
// logd of it, as hexadecimal doubles.
#include <hip/hip_runtime.h>

#include <cstdio>

thread_local emu_dim3 emu_threadIdx;
int emu_dpp(int x, int) { return x; }
unsigned long long emu_shfl_xor(unsigned long long x, int) { return x; }

#include "../../paper_1701_05431_amd/csrc/fvm_internal.hpp"
#include "../../paper_1701_05431_amd/csrc/fvm_models.hpp"

int main() {
  double x;
  while (std::scanf("%la", &x) == 1) std::printf("%a %a\n", x, fvm::logd(x));
  return 0;
}
