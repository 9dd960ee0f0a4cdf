// Host stand-in for <hip/hip_runtime.h>, used only by the CPU emulators in
// tests/emu (strip_emu.cpp, adjoint_emu.cpp, spray_adjoint_emu.cpp): it lets
// the device headers compile as plain C++ so that the 64 lanes of a wave run
// as 64 host threads in lockstep (or, for the spray adjoint's per-thread
// code, one thread after another). Cross-lane moves (DPP
// row shifts, xor shuffles) go through a shared slot array between two
// barriers; the hardware reciprocal / rsqrt estimates become exact host
// arithmetic. The reduction atomics are single-threaded stand-ins: the
// harness never calls the code that uses them.
#pragma once
#include <algorithm>
#include <barrier>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstring>

#define __device__
#define __host__
#define __global__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static

struct emu_dim3 {
  unsigned x, y, z;
};
extern thread_local emu_dim3 emu_threadIdx;
#define threadIdx emu_threadIdx

using std::exp;
using std::fabs;
using std::fma;
using std::frexp;
using std::log;
using std::sqrt;
inline int min(int a, int b) { return a < b ? a : b; }
inline int max(int a, int b) { return a > b ? a : b; }
inline long long __double_as_longlong(double x) {
  long long r;
  std::memcpy(&r, &x, 8);
  return r;
}
inline double __longlong_as_double(long long x) {
  double r;
  std::memcpy(&r, &x, 8);
  return r;
}

// lane exchanges of the wave the calling thread belongs to (strip_emu.cpp)
int emu_dpp(int x, int ctrl);
unsigned long long emu_shfl_xor(unsigned long long x, int o);
#define __builtin_amdgcn_update_dpp(old, x, ctrl, rm, bm, bc) emu_dpp((x), (ctrl))
#define __builtin_amdgcn_readfirstlane(x) (x)
// FVM_EMU_EST_ERR: a relative error given to both estimates, to exercise
// the refinement steps that follow them in the device code
#ifndef FVM_EMU_EST_ERR
#define FVM_EMU_EST_ERR 0.0
#endif
#define __builtin_amdgcn_rcp(x) ((1.0 / (x)) * (1.0 + FVM_EMU_EST_ERR))
#define __builtin_amdgcn_rsq(x) ((1.0 / std::sqrt(x)) * (1.0 + FVM_EMU_EST_ERR))
template <class T>
inline T __shfl_xor(T x, int o, int) {
  return (T)emu_shfl_xor((unsigned long long)x, o);
}

template <class T, class U>
inline T atomicExch(T* p, U v) {
  T o = *p;
  *p = (T)v;
  return o;
}
template <class T, class U>
inline T atomicOr(T* p, U v) {
  T o = *p;
  *p = o | (T)v;
  return o;
}
template <class T, class U>
inline T atomicMax(T* p, U v) {
  T o = *p;
  if ((T)v > o) *p = (T)v;
  return o;
}
template <class T, class U>
inline T atomicAdd(T* p, U v) {
  T o = *p;
  *p = o + (T)v;
  return o;
}
inline void __threadfence() {}
inline void __syncthreads() {}

typedef int hipError_t;
typedef void* hipStream_t;
