// trs_membench.hip -- memory microbenchmarks of the device, the method of the
// paper's hardware comparison (Section 4, the table of aligned and random
// bandwidths) re-done for the MI355X, plus the latencies that bound one
// rewrite round: a dependent chain of loads and of returning atomics.
#include <hip/hip_runtime.h>

#include <cstring>

#include "trs.h"

namespace {

__device__ __forceinline__ uint32_t mix32(uint32_t x) {
  // integer hash (multiply-xorshift), used only to spread indices
  x ^= x >> 16;
  x *= 0x7feb352dU;
  x ^= x >> 15;
  x *= 0x846ca68bU;
  x ^= x >> 16;
  return x;
}

__global__ void k_fill(uint32_t *a, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    a[i] = (uint32_t)i;
}

// coalesced streaming read of n uint4
__global__ void k_stream(const uint4 *a, size_t n, uint32_t *sink) {
  uint32_t acc = 0;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    const uint4 v = a[i];
    acc ^= v.x ^ v.y ^ v.z ^ v.w;
  }
  if (acc == 0x12345678u) sink[0] = acc;
}

// k random 4-byte reads per thread from an array of n words
__global__ void k_gather4(const uint32_t *a, size_t n, int k, uint32_t *sink) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t acc = 0;
  for (int j = 0; j < k; j++) acc ^= a[mix32(t * 977u + j * 7919u) % n];
  if (acc == 0x12345678u) sink[0] = acc;
}

// k random 1-byte reads per thread from an array of n bytes
__global__ void k_gather1(const uint8_t *a, size_t n, int k, uint32_t *sink) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t acc = 0;
  for (int j = 0; j < k; j++) acc += a[mix32(t * 977u + j * 7919u) % n];
  if (acc == 0x12345678u) sink[0] = acc;
}

// k random atomic increments (no return) per thread over n words
__global__ void k_atomics(uint32_t *a, size_t n, int k) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  for (int j = 0; j < k; j++) atomicAdd(&a[mix32(t * 977u + j * 7919u) % n], 1u);
}

// one wave follows 64 independent chains of dependent loads through a[]
// (each value is the next index): per-lane addresses keep the loads on the
// vector memory path; the time per step is one load latency
__global__ void k_chase(const uint32_t *a, int steps, uint32_t start, uint32_t n,
                        uint32_t *out) {
  uint32_t i = (start + threadIdx.x * 4099u) % n;  // on the cycle of length n
  for (int j = 0; j < steps; j++) i = a[i];
  out[threadIdx.x] = i;
}

// one wave performs 64 independent chains of dependent returning atomics:
// the address of each depends on the value returned by the previous one
__global__ void k_atomic_chain(uint32_t *a, size_t n, int steps, uint32_t *out) {
  uint32_t i = (threadIdx.x * 977u) % n;
  for (int j = 0; j < steps; j++) {
    const uint32_t v = atomicAdd(&a[i], 1u);
    i = mix32(v + j + threadIdx.x) % n;
  }
  out[threadIdx.x] = i;
}

// plain copy of n uint4 (calibrates the memory counters: n*16 bytes read
// and n*16 bytes written)
__global__ void k_copy(const uint4 *a, uint4 *b, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}

}  // namespace

extern "C" trs_status trs_membench(int32_t device, trs_membench_result *out) {
  if (!out) return TRS_E_ARG;
  std::memset(out, 0, sizeof(*out));
  if (hipSetDevice(device) != hipSuccess) return TRS_E_HIP;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return TRS_E_HIP;
  out->cu_count = prop.multiProcessorCount;
  out->clock_mhz = prop.clockRate / 1000.0;
  out->l2_bytes = prop.l2CacheSize;
  hipStream_t s;
  if (hipStreamCreate(&s) != hipSuccess) return TRS_E_HIP;
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  const size_t big = (size_t)2 << 30;  // 2 GiB: well beyond the 256 MB last-level cache
  const size_t small1 = (size_t)64 << 20;  // 64 MiB: resident in the last-level cache
  uint32_t *a = nullptr, *sink = nullptr;
  if (hipMalloc(&a, big) != hipSuccess) return TRS_E_HIP;
  if (hipMalloc(&sink, 256) != hipSuccess) {
    (void)hipFree(a);
    return TRS_E_HIP;
  }
  const size_t nw = big / 4;
  const int G = prop.multiProcessorCount * 16, B = 256;
  hipLaunchKernelGGL(k_fill, dim3(G), dim3(B), 0, s, a, nw);
  auto timed = [&](auto launch, int reps) {
    launch();  // warm
    (void)hipEventRecord(e0, s);
    for (int i = 0; i < reps; i++) launch();
    (void)hipEventRecord(e1, s);
    (void)hipEventSynchronize(e1);
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    return ms / reps;
  };
  // stream
  float ms = timed([&] { hipLaunchKernelGGL(k_stream, dim3(G), dim3(B), 0, s, (const uint4 *)a, big / 16, sink); }, 5);
  out->stream_read_gbps = big / (ms * 1e-3) / 1e9;
  // random 4-byte gathers over 2 GiB and over 64 MiB
  const int K = 16;
  const size_t threads = (size_t)G * B;
  ms = timed([&] { hipLaunchKernelGGL(k_gather4, dim3(G), dim3(B), 0, s, (const uint32_t *)a, nw, K, sink); }, 5);
  out->gather4_hbm_gops = threads * K / (ms * 1e-3) / 1e9;
  ms = timed([&] { hipLaunchKernelGGL(k_gather4, dim3(G), dim3(B), 0, s, (const uint32_t *)a, small1 / 4, K, sink); }, 5);
  out->gather4_llc_gops = threads * K / (ms * 1e-3) / 1e9;
  ms = timed([&] { hipLaunchKernelGGL(k_gather1, dim3(G), dim3(B), 0, s, (const uint8_t *)a, small1, K, sink); }, 5);
  out->gather1_llc_gops = threads * K / (ms * 1e-3) / 1e9;
  // random atomics (no return) over 512 MiB
  ms = timed([&] { hipLaunchKernelGGL(k_atomics, dim3(G), dim3(B), 0, s, a, (size_t)128 << 20, K); }, 3);
  out->atomic_random_gops = threads * K / (ms * 1e-3) / 1e9;
  // latency: dependent loads through a single random cycle (Sattolo's
  // shuffle, built on the host) over 512 MiB (misses every cache) and over
  // 256 KiB (L2 hits)
  {
    const size_t nchase = (size_t)128 << 20;  // words (512 MiB)
    uint32_t *h = (uint32_t *)malloc(nchase * 4);
    if (h) {
      for (size_t i = 0; i < nchase; i++) h[i] = (uint32_t)i;
      uint64_t x = 0x9e3779b97f4a7c15ull;
      for (size_t i = nchase - 1; i > 0; i--) {  // Sattolo: one cycle
        x ^= x << 13;
        x ^= x >> 7;
        x ^= x << 17;
        size_t j = x % i;
        uint32_t t = h[i];
        h[i] = h[j];
        h[j] = t;
      }
      (void)hipMemcpy(a, h, nchase * 4, hipMemcpyHostToDevice);
      const int steps = 20000;
      ms = timed([&] { hipLaunchKernelGGL(k_chase, dim3(1), dim3(64), 0, s, (const uint32_t *)a, steps, 1u, (uint32_t)nchase, sink); }, 2);
      out->load_latency_far_ns = ms * 1e6 / steps;
      const size_t nsm = 64 << 10;  // 256 KiB
      for (size_t i = 0; i < nsm; i++) h[i] = (uint32_t)i;
      for (size_t i = nsm - 1; i > 0; i--) {
        x ^= x << 13;
        x ^= x >> 7;
        x ^= x << 17;
        size_t j = x % i;
        uint32_t t = h[i];
        h[i] = h[j];
        h[j] = t;
      }
      (void)hipMemcpy(a, h, nsm * 4, hipMemcpyHostToDevice);
      ms = timed([&] { hipLaunchKernelGGL(k_chase, dim3(1), dim3(64), 0, s, (const uint32_t *)a, steps, 1u, (uint32_t)nsm, sink); }, 2);
      out->load_latency_near_ns = ms * 1e6 / steps;
      free(h);
    }
    const int asteps = 5000;
    ms = timed([&] { hipLaunchKernelGGL(k_atomic_chain, dim3(1), dim3(64), 0, s, a, (size_t)64 << 10, asteps, sink); }, 2);
    out->atomic_latency_ns = ms * 1e6 / asteps;
  }
  // copy of 256 MiB into a second buffer (the upper half of the 2 GiB block)
  {
    const size_t cb = (size_t)256 << 20;
    uint4 *src = (uint4 *)a, *dst = (uint4 *)((char *)a + ((size_t)1 << 30));
    ms = timed([&] { hipLaunchKernelGGL(k_copy, dim3(G), dim3(B), 0, s, (const uint4 *)src, dst, cb / 16); }, 5);
    out->copy_gbps = 2.0 * cb / (ms * 1e-3) / 1e9;
    out->copy_bytes = (int64_t)cb;
  }
  // launch: an empty chain of small kernels
  ms = timed([&] { hipLaunchKernelGGL(k_chase, dim3(1), dim3(1), 0, s, (const uint32_t *)a, 0, 0u, 1u, sink); }, 200);
  out->empty_kernel_us = ms * 1e3;
  (void)hipStreamSynchronize(s);
  (void)hipFree(a);
  (void)hipFree(sink);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamDestroy(s);
  return TRS_OK;
}
