// logd_emu.cpp -- the kernels' logarithm and reciprocal square root
// (fvm_models.hpp, logd and rroot) built for the host: prints, for each
// argument read from stdin, the argument and the function (argv[1]: "logd"
// or "rroot") of it, as hexadecimal doubles.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>

thread_local emu_dim3 emu_threadIdx;
int emu_dpp(int x, int) { return x; }
unsigned long long emu_shfl_xor(unsigned long long x, int) { return x; }

#include "../../paper_1701_05431_amd/csrc/fvm_internal.hpp"
#include "../../paper_1701_05431_amd/csrc/fvm_models.hpp"

int main(int argc, char** argv) {
  if (argc != 2) return 2;
  const bool root = std::strcmp(argv[1], "rroot") == 0;
  if (!root && std::strcmp(argv[1], "logd") != 0) return 2;
  double x;
  while (std::scanf("%la", &x) == 1)
    std::printf("%a %a\n", x, root ? fvm::rroot(x) : fvm::logd(x));
  return 0;
}
