// lc_probe.hip -- measurement probes that set the ceilings the loop-cluster
// kernels are measured against on this device: a device-to-device streaming
// copy (HBM bandwidth) and random 8-byte compare-and-swap on a word array
// (the access pattern of a lock-free union-find hook, Sec. 3.2), once on an
// array far larger than the caches and once on one that stays in L2.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <new>

#include "lc.h"

namespace {

constexpr int kProbeBlock = 256;

// splitmix64 finaliser (Steele, Lea, Flood, "Fast splittable pseudorandom
// number generators", OOPSLA 2014): a bijective 64-bit mixer.
__device__ inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ __launch_bounds__(kProbeBlock) void k_probe_fill(unsigned long long* __restrict__ a,
                                                            int64_t n) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kProbeBlock + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kProbeBlock)
    a[i] = static_cast<unsigned long long>(i);
}

// Every thread issues `per_thread` compare-and-swaps on words chosen by the
// mixer; each compares with the word's index, which it holds, so every CAS
// succeeds and leaves the array unchanged (an atomic read-modify-write of a
// random line).  Successes are counted per thread into `hits` (vector store).
__global__ __launch_bounds__(kProbeBlock) void k_probe_cas(unsigned long long* __restrict__ a,
                                                           uint64_t mask, int per_thread,
                                                           uint64_t salt,
                                                           unsigned int* __restrict__ hits) {
  const uint64_t t = static_cast<uint64_t>(blockIdx.x) * kProbeBlock + threadIdx.x;
  unsigned int ok = 0;
  for (int r = 0; r < per_thread; ++r) {
    const uint64_t i = mix64(salt + t * 0x9E3779B97F4A7C15ull + static_cast<uint64_t>(r)) & mask;
    const unsigned long long old = atomicCAS(a + i, static_cast<unsigned long long>(i),
                                             static_cast<unsigned long long>(i));
    ok += old == i ? 1u : 0u;
  }
  hits[t] = ok;
}

__global__ __launch_bounds__(kProbeBlock) void k_probe_copy(const uint4* __restrict__ src,
                                                            uint4* __restrict__ dst, int64_t n) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kProbeBlock + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kProbeBlock)
    dst[i] = src[i];
}

int status(hipError_t e) { return e == hipSuccess ? LC_OK : LC_EDEVICE; }

}  // namespace

extern "C" int lc_probe_cas(int log2_words, int64_t n_cas, int repeats, void* hip_stream,
                            double* cas_per_s, double* success_frac) {
  if (log2_words < 10 || log2_words > 34 || n_cas < kProbeBlock || repeats < 1 || !cas_per_s)
    return LC_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const int64_t words = int64_t(1) << log2_words;
  const int per_thread = 16;
  const int64_t threads = (n_cas / per_thread + kProbeBlock - 1) / kProbeBlock * kProbeBlock;
  const int blocks = static_cast<int>(threads / kProbeBlock);
  unsigned long long* a = nullptr;
  unsigned int* hits = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = LC_OK;
  if (hipMalloc(&a, words * sizeof(unsigned long long)) != hipSuccess) return LC_ENOMEM;
  if (hipMalloc(&hits, threads * sizeof(unsigned int)) != hipSuccess) {
    (void)hipFree(a);
    return LC_ENOMEM;
  }
  float best = 0.f;
  if ((rc = status(hipEventCreate(&e0))) == LC_OK && (rc = status(hipEventCreate(&e1))) == LC_OK) {
    hipLaunchKernelGGL(k_probe_fill, dim3(4096), dim3(kProbeBlock), 0, s, a, words);
    for (int r = 0; r <= repeats && rc == LC_OK; ++r) {  // launch 0 warms up
      (void)hipEventRecord(e0, s);
      hipLaunchKernelGGL(k_probe_cas, dim3(blocks), dim3(kProbeBlock), 0, s, a,
                         static_cast<uint64_t>(words - 1), per_thread,
                         static_cast<uint64_t>(r) * 0x632BE59BD9B4E019ull, hits);
      (void)hipEventRecord(e1, s);
      float ms = 0.f;
      if ((rc = status(hipEventSynchronize(e1))) != LC_OK) break;
      if ((rc = status(hipEventElapsedTime(&ms, e0, e1))) != LC_OK) break;
      if (r > 0 && (best == 0.f || ms < best)) best = ms;
    }
  }
  if (rc == LC_OK) {
    const double total = static_cast<double>(threads) * per_thread;
    *cas_per_s = total / (static_cast<double>(best) * 1e-3);
    if (success_frac) {
      unsigned int* h = new (std::nothrow) unsigned int[threads];
      if (!h) {
        rc = LC_ENOMEM;
      } else {
        if (hipMemcpy(h, hits, threads * sizeof(unsigned int), hipMemcpyDeviceToHost) != hipSuccess)
          rc = LC_EDEVICE;
        double ok = 0;
        for (int64_t i = 0; i < threads; ++i) ok += h[i];
        *success_frac = ok / total;
        delete[] h;
      }
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(hits);
  (void)hipFree(a);
  return rc;
}

extern "C" int lc_probe_copy(int64_t bytes, int repeats, void* hip_stream, double* gb_per_s) {
  if (bytes < (1 << 20) || repeats < 1 || !gb_per_s) return LC_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const int64_t n = bytes / 16;
  uint4 *src = nullptr, *dst = nullptr;
  if (hipMalloc(&src, n * 16) != hipSuccess) return LC_ENOMEM;
  if (hipMalloc(&dst, n * 16) != hipSuccess) {
    (void)hipFree(src);
    return LC_ENOMEM;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = status(hipMemsetAsync(src, 1, n * 16, s));
  float best = 0.f;
  if (rc == LC_OK && (rc = status(hipEventCreate(&e0))) == LC_OK &&
      (rc = status(hipEventCreate(&e1))) == LC_OK) {
    for (int r = 0; r <= repeats && rc == LC_OK; ++r) {
      (void)hipEventRecord(e0, s);
      hipLaunchKernelGGL(k_probe_copy, dim3(8192), dim3(kProbeBlock), 0, s, src, dst, n);
      (void)hipEventRecord(e1, s);
      float ms = 0.f;
      if ((rc = status(hipEventSynchronize(e1))) != LC_OK) break;
      if ((rc = status(hipEventElapsedTime(&ms, e0, e1))) != LC_OK) break;
      if (r > 0 && (best == 0.f || ms < best)) best = ms;
    }
  }
  if (rc == LC_OK) *gb_per_s = 2.0 * static_cast<double>(n) * 16 / (static_cast<double>(best) * 1e-3) / 1e9;
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(src);
  (void)hipFree(dst);
  return rc;
}
