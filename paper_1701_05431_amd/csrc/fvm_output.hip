// fvm_output.hip -- asynchronous solution output (Sec. 4.3).
//
// The paper dumps the solution without a global synchronisation: each
// subdomain copies its part into its block of one contiguous output buffer
// (per-part views of the global buffer through a leading dimension), the
// buffer is then switched to a single global handle and one task writes it to
// disk while the time steps go on. Here the per-part copies are one gather
// kernel over the whole grid, enqueued on the grid's stream in order with the
// steps (the next step may overwrite the state only after it); the switch to
// the global buffer is the stream order itself; the device-to-host copy runs
// on a second stream and a host thread of the stage writes the file, so the
// grid's stream never waits for PCIe or the disk. One staging buffer and one
// host buffer: a snapshot waits (on the host) only while the previous one is
// still being written.
#include <hip/hip_runtime.h>

#include <condition_variable>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <thread>

#include "../../include/fvm.h"
#include "fvm_host.hpp"
#include "fvm_internal.hpp"

namespace fvm {

constexpr int kGatherThreads = 256;
constexpr int kGatherPer = 8;                            // doubles in flight per thread
constexpr int kGatherSeg = kGatherThreads * kGatherPer;  // columns per workgroup

struct GatherArgs {
  const double* src;
  double* dst;
  size_t plane;  // variable stride of the state
  int ld;        // grid-row stride of one variable
  int nx, ny;
  int nseg;      // workgroups per row
};

// Workgroup b copies columns [seg * kGatherSeg, ...) of output row r =
// v * ny + j: all loads of a thread are issued before its stores.
__global__ __launch_bounds__(kGatherThreads) void gather_kernel(GatherArgs a) {
  const long long b = blockIdx.x;
  const int seg = static_cast<int>(b % a.nseg);
  const long long r = b / a.nseg;
  const int v = static_cast<int>(r / a.ny), j = static_cast<int>(r % a.ny);
  const double* s = a.src + v * a.plane + static_cast<size_t>(j) * a.ld;
  double* d = a.dst + static_cast<size_t>(r) * a.nx;
  const int i0 = seg * kGatherSeg + static_cast<int>(threadIdx.x);
  double x[kGatherPer];
#pragma unroll
  for (int k = 0; k < kGatherPer; ++k) {
    const int i = i0 + k * kGatherThreads;
    x[k] = i < a.nx ? s[i] : 0.0;
  }
#pragma unroll
  for (int k = 0; k < kGatherPer; ++k) {
    const int i = i0 + k * kGatherThreads;
    if (i < a.nx) d[i] = x[k];
  }
}

static hipError_t launch_gather(const GridView& v, double* dst) {
  GatherArgs a{};
  a.src = v.cur;
  a.dst = dst;
  a.plane = v.g.plane;
  a.ld = v.g.ld;
  a.nx = v.g.nx;
  a.ny = v.g.ny;
  a.nseg = (v.g.nx + kGatherSeg - 1) / kGatherSeg;
  const long long blocks = static_cast<long long>(a.nseg) * v.nv * v.g.ny;
  if (blocks < 1 || blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(gather_kernel, dim3(static_cast<unsigned>(blocks)), dim3(kGatherThreads),
                     0, v.stream, a);
  return hipGetLastError();
}

}  // namespace fvm

using namespace fvm;

struct fvm_output {
  fvm_grid* grid = nullptr;
  double* staging = nullptr;
  double* host = nullptr;
  hipStream_t cs = nullptr;
  size_t n = 0;  // doubles per snapshot
  int nx = 0, ny = 0, nv = 0;
  hipEvent_t gathered = nullptr, copied = nullptr;
  std::thread writer;
  std::mutex mu;
  std::condition_variable cv;
  bool pending = false;  // a snapshot holds the host buffer (copy or write in progress)
  bool stop = false;
  int err = FVM_OK;
  std::string path;
  unsigned char header[64] = {};

  void run() {
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      cv.wait(lk, [&] { return stop || pending; });
      if (!pending) return;  // stop with nothing left to write
      const std::string p = path;
      unsigned char h[64];
      std::memcpy(h, header, sizeof h);
      lk.unlock();
      int rc = hipEventSynchronize(copied) == hipSuccess ? FVM_OK : FVM_EDEVICE;
      if (rc == FVM_OK) {
        std::FILE* f = std::fopen(p.c_str(), "wb");
        if (!f) {
          rc = FVM_EIO;
        } else {
          if (std::fwrite(h, 1, sizeof h, f) != sizeof h ||
              std::fwrite(host, sizeof(double), n, f) != n)
            rc = FVM_EIO;
          if (std::fclose(f) != 0) rc = FVM_EIO;
        }
      }
      lk.lock();
      if (rc != FVM_OK && err == FVM_OK) err = rc;
      pending = false;
      cv.notify_all();
    }
  }
};

extern "C" {

int fvm_output_create(fvm_grid* g, double* staging, double* host, void* copy_stream,
                      fvm_output** out) {
  if (!out) return FVM_EINVAL;
  *out = nullptr;
  GridView v{};
  if (!g || !staging || !host || grid_view(g, &v) != FVM_OK) return FVM_EINVAL;
  if (static_cast<hipStream_t>(copy_stream) == v.stream) return FVM_EINVAL;
  fvm_output* o = new (std::nothrow) fvm_output();
  if (!o) return FVM_EINVAL;
  o->grid = g;
  o->staging = staging;
  o->host = host;
  o->cs = static_cast<hipStream_t>(copy_stream);
  o->nx = v.g.nx;
  o->ny = v.g.ny;
  o->nv = v.nv;
  o->n = static_cast<size_t>(v.nv) * v.g.ny * v.g.nx;
  if (hipEventCreateWithFlags(&o->gathered, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&o->copied, hipEventDisableTiming) != hipSuccess) {
    if (o->gathered) (void)hipEventDestroy(o->gathered);
    delete o;
    return FVM_EDEVICE;
  }
  o->writer = std::thread([o] { o->run(); });
  *out = o;
  return FVM_OK;
}

int fvm_output_snapshot(fvm_output* o, const char* path, long long step, double time) {
  if (!o || !path || !*path) return FVM_EINVAL;
  {
    std::unique_lock<std::mutex> lk(o->mu);
    o->cv.wait(lk, [&] { return !o->pending; });
    if (o->err != FVM_OK) return o->err;
  }
  GridView v{};
  if (grid_view(o->grid, &v) != FVM_OK) return FVM_EINVAL;
  if (v.g.nx != o->nx || v.g.ny != o->ny || v.nv != o->nv) return FVM_EINVAL;
  if (launch_gather(v, o->staging) != hipSuccess) return FVM_EDEVICE;
  if (hipEventRecord(o->gathered, v.stream) != hipSuccess ||
      hipStreamWaitEvent(o->cs, o->gathered, 0) != hipSuccess ||
      hipMemcpyAsync(o->host, o->staging, sizeof(double) * o->n, hipMemcpyDeviceToHost,
                     o->cs) != hipSuccess ||
      hipEventRecord(o->copied, o->cs) != hipSuccess)
    return FVM_EDEVICE;
  unsigned char h[64] = {};
  std::memcpy(h, "FVMSNAP1", 8);
  const int32_t ints[4] = {v.p.model, v.nv, v.g.nx, v.g.ny};
  std::memcpy(h + 8, ints, sizeof ints);
  const int64_t st = step;
  std::memcpy(h + 24, &st, 8);
  const double dbl[3] = {time, v.p.lx, v.p.ly};
  std::memcpy(h + 32, dbl, sizeof dbl);
  const int32_t parts[2] = {v.p.npart_x, v.p.npart_y};
  std::memcpy(h + 56, parts, sizeof parts);
  {
    std::lock_guard<std::mutex> lk(o->mu);
    o->path = path;
    std::memcpy(o->header, h, sizeof h);
    o->pending = true;
  }
  o->cv.notify_all();
  return FVM_OK;
}

int fvm_output_wait(fvm_output* o) {
  if (!o) return FVM_EINVAL;
  std::unique_lock<std::mutex> lk(o->mu);
  o->cv.wait(lk, [&] { return !o->pending; });
  return o->err;
}

int fvm_output_destroy(fvm_output* o) {
  if (!o) return FVM_OK;
  const int rc = fvm_output_wait(o);
  {
    std::lock_guard<std::mutex> lk(o->mu);
    o->stop = true;
  }
  o->cv.notify_all();
  if (o->writer.joinable()) o->writer.join();
  (void)hipEventDestroy(o->gathered);
  (void)hipEventDestroy(o->copied);
  delete o;
  return rc;
}

}  // extern "C"
