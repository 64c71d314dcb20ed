// Micro-benchmark: global float atomic and random-load throughput on gfx950
// (the measurement behind binning the encoding's gradient instead of
// scattering it with atomics).  1 M threads x 16 operations on a buffer of
// 64 MiB; every index is masked into the buffer.
//   hipcc --offload-arch=gfx950 -O3 -munsafe-fp-atomics \
//         -Xclang -target-feature -Xclang -packed-fp32-ops -o global_atomics global_atomics.hip
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdint>
#include <vector>
#include <cmath>

#define CHK(x) do { hipError_t e = (x); if (e != hipSuccess) { printf("HIP %s at %d\n", hipGetErrorString(e), __LINE__); return 1; } } while (0)

__device__ inline uint32_t hash32(uint32_t x) { x ^= x >> 16; x *= 0x7feb352du; x ^= x >> 15; x *= 0x846ca68bu; x ^= x >> 16; return x; }

__global__ void k_atomic_rand(float* buf, uint32_t mask, int64_t n, int per_thread) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  for (int k = 0; k < per_thread; ++k) {
    uint32_t i = hash32((uint32_t)(t * per_thread + k)) & mask;
    unsafeAtomicAdd(buf + i, 1.0f);
  }
}
__global__ void k_atomic_rand_wg(float* buf, uint32_t mask, int64_t n, int per_thread) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  for (int k = 0; k < per_thread; ++k) {
    uint32_t i = hash32((uint32_t)(t * per_thread + k)) & mask;
    __hip_atomic_fetch_add(buf + i, 1.0f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
}
__global__ void k_load_rand(const float* buf, float* out, uint32_t mask, int64_t n, int per_thread) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  float s = 0;
  for (int k = 0; k < per_thread; ++k) {
    uint32_t i = hash32((uint32_t)(t * per_thread + k)) & mask;
    s += buf[i];
  }
  if (s == 12345.0f) out[0] = s;
}
// contiguous (coalesced) atomics: each wave hits 64 consecutive floats
__global__ void k_atomic_coal(float* buf, uint32_t mask, int64_t n, int per_thread) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  for (int k = 0; k < per_thread; ++k) {
    uint32_t base = (hash32((uint32_t)((t >> 6) * per_thread + k)) << 6);
    uint32_t i = (base + (uint32_t)(t & 63)) & mask;
    unsafeAtomicAdd(buf + i, 1.0f);
  }
}

int main() {
  const int64_t nthreads = 1 << 20;  // 1M threads
  const int per = 16;                // 16M atomics
  float* buf; float* out;
  CHK(hipMalloc(&buf, (size_t)64 << 20));
  CHK(hipMalloc(&out, 64));
  CHK(hipMemset(buf, 0, (size_t)64 << 20));
  hipEvent_t a, b; CHK(hipEventCreate(&a)); CHK(hipEventCreate(&b));
  struct Case { const char* name; int kind; uint32_t mask; };
  Case cases[] = {
    {"atomic agent rand 64KB", 0, (1u << 14) - 1},
    {"atomic agent rand 4MB", 0, (1u << 20) - 1},
    {"atomic agent rand 32MB", 0, (1u << 23) - 1},
    {"atomic wg rand 4MB", 1, (1u << 20) - 1},
    {"atomic wg rand 64KB", 1, (1u << 14) - 1},
    {"load rand 4MB", 2, (1u << 20) - 1},
    {"load rand 32MB", 2, (1u << 23) - 1},
    {"atomic agent coalesced 4MB", 3, (1u << 20) - 1},
    {"atomic agent coalesced 32MB", 3, (1u << 23) - 1},
  };
  for (auto& c : cases) {
    for (int rep = 0; rep < 3; ++rep) {
      CHK(hipEventRecord(a));
      dim3 g((unsigned)(nthreads / 256)), bl(256);
      if (c.kind == 0) k_atomic_rand<<<g, bl>>>(buf, c.mask, nthreads, per);
      if (c.kind == 1) k_atomic_rand_wg<<<g, bl>>>(buf, c.mask, nthreads, per);
      if (c.kind == 2) k_load_rand<<<g, bl>>>(buf, out, c.mask, nthreads, per);
      if (c.kind == 3) k_atomic_coal<<<g, bl>>>(buf, c.mask, nthreads, per);
      CHK(hipGetLastError());
      CHK(hipEventRecord(b));
      CHK(hipEventSynchronize(b));
      float ms; CHK(hipEventElapsedTime(&ms, a, b));
      if (rep == 2) printf("%-30s %8.3f ms  %7.1f G ops/s\n", c.name, ms, nthreads * per / (ms * 1e6));
    }
  }
  return 0;
}
