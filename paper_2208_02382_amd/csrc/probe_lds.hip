// Throughput of 64-bit integer LDS atomics (ds_add_u64) on this GPU, the operation the binned
// charge deposit is built on: a reference figure that the bench reports next to the deposit's
// achieved atomic rate.  Not part of libpic.so.
//
// Every lane adds 1 to a window of 8-byte counters in LDS, `iters` times.  Pattern 0: lane l of
// a wave hits word (l + 64 q) of its wave's 4 KB stripe (consecutive words, no bank conflict);
// pattern 1: every lane hits a word picked by a multiplicative hash of (thread, q) in one
// shared 32 KB window (a scattered pattern, as the deposit's lanes in unrelated cells
// produce).  All addresses stay inside the LDS array.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

constexpr int kWords = 4096;  // 32 KB of counters per workgroup

template <int PATTERN>
__global__ __launch_bounds__(1024) void k_lds_atomics(int iters, unsigned long long* sink) {
  __shared__ unsigned long long win[kWords];
  for (int w = threadIdx.x; w < kWords; w += blockDim.x) win[w] = 0ull;
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int q = 0; q < iters; ++q) {
    int w;
    if (PATTERN == 0)
      w = (wave * 512 + lane + 64 * (q & 7)) & (kWords - 1);
    else
      w = (int)(((uint32_t)threadIdx.x * 2654435761u + (uint32_t)q * 2246822519u) >> 20) &
          (kWords - 1);
    atomicAdd(&win[w], 1ull);
  }
  __syncthreads();
  // keep the result observable: one global write per workgroup
  if (threadIdx.x == 0) sink[blockIdx.x] = win[blockIdx.x & (kWords - 1)];
}

}  // namespace

extern "C" int probe_lds_u64_atomics(int pattern, int blocks, int threads, int iters,
                                     double* ms_out) {
  if (blocks < 1 || threads < 64 || threads > 1024 || (threads & 63) || iters < 1 || !ms_out)
    return -1;
  unsigned long long* sink = nullptr;
  if (hipMalloc(&sink, sizeof(unsigned long long) * blocks) != hipSuccess) return -2;
  hipEvent_t a, b;
  hipEventCreate(&a);
  hipEventCreate(&b);
  auto launch = [&]() {
    if (pattern == 0)
      hipLaunchKernelGGL(k_lds_atomics<0>, dim3(blocks), dim3(threads), 0, 0, iters, sink);
    else
      hipLaunchKernelGGL(k_lds_atomics<1>, dim3(blocks), dim3(threads), 0, 0, iters, sink);
  };
  launch();  // warm-up
  hipEventRecord(a, 0);
  launch();
  hipEventRecord(b, 0);
  hipEventSynchronize(b);
  float ms = 0.0f;
  hipEventElapsedTime(&ms, a, b);
  hipError_t e = hipGetLastError();
  hipEventDestroy(a);
  hipEventDestroy(b);
  hipFree(sink);
  *ms_out = ms;
  return e == hipSuccess ? 0 : -3;
}
