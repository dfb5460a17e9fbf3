// pic_moments_noalloc: the beam statistics of pic_moments for callers that cannot allocate
// device memory (code under HIP graph capture, serving loops, harnesses that forbid it).
//
// The reduction's per-block partial sums live in a file-scope device array instead of a
// workspace.  Host code never passes that array's name to a kernel (on the host it is only a
// stand-in for the registered symbol): its device address is looked up once per device with
// hipGetSymbolAddress and kept, and the kernels take that address.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/pic.h"
#include "internal.hpp"

using namespace pic;

namespace {

// partial sums of the two reduction passes: kReduceBlocks blocks x kMomentSlots slots (221 KB);
// every launch writes all of them before they are read, so nothing needs clearing
constexpr size_t kScratchDoubles = (size_t)kReduceBlocks * kMomentSlots;
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_scratch[kMaxDevices];  // device address of `scratch` on each device, once looked up

// the device address of `scratch` on the current device (looked up on the first call there)
hipError_t scratch_ptr(double** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[dev] = (double*)p;
  }
  *out = g_scratch[dev];
  return hipSuccess;
}

}  // namespace

extern "C" pic_status pic_moments_noalloc(const double* d_X, int64_t n, double* d_out,
                                          void* stream) {
  if (!d_X || !d_out) return (pic_status)record_failure(PIC_EINVAL, "NULL argument");
  if (((uintptr_t)d_X | (uintptr_t)d_out) & 7)
    return (pic_status)record_failure(PIC_EINVAL, "X and out must be 8-byte aligned");
  if (n < 1 || n > 0x7fffffffLL)
    return (pic_status)record_failure(PIC_EINVAL, "n must be in 1 .. 2^31 - 1");
  double* partial = nullptr;
  hipError_t e = scratch_ptr(&partial);
  if (e == hipSuccess) e = launch_moments(d_X, n, partial, d_out, (hipStream_t)stream);
  if (e != hipSuccess) return (pic_status)record_hip_failure(e, "pic_moments_noalloc");
  return PIC_OK;
}
