// Micro-benchmark: LDS atomic throughput on gfx950 (the measurement behind the
// fixed-point region sums of k_bin_acc).  2048 workgroups of 512 threads each
// do 1024 LDS operations per thread on a 64 KiB image; every address is masked
// into the image.  Prints lane-operations per second and per CU clock.
//   hipcc --offload-arch=gfx950 -O3 -munsafe-fp-atomics \
//         -Xclang -target-feature -Xclang -packed-fp32-ops -o lds_atomics lds_atomics.hip
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdint>
#include <cstdlib>
#define CHK(x) do { hipError_t e = (x); if (e != hipSuccess) { printf("HIP %s at %d\n", hipGetErrorString(e), __LINE__); exit(1); } } while (0)
constexpr int WORDS = 16384;  // 64 KiB of 32-bit words
constexpr int ITERS = 1024;

__device__ inline uint32_t h32(uint32_t x) { x ^= x >> 16; x *= 0x7feb352du; x ^= x >> 15; x *= 0x846ca68bu; x ^= x >> 16; return x; }

template <int MODE>
__global__ __launch_bounds__(512) void k_lds(float* out) {
  __shared__ uint32_t img[WORDS];
  for (int e = threadIdx.x; e < WORDS; e += 512) img[e] = 0;
  __syncthreads();
  uint32_t a = h32(threadIdx.x * 977u + blockIdx.x * 7919u);
  for (int i = 0; i < ITERS; ++i) {
    a = a * 1664525u + 1013904223u;  // LCG: cheap per-lane pseudo-random
    uint32_t w;
    if (MODE == 2 || MODE == 3) w = (threadIdx.x + 512u * (uint32_t)i) & (WORDS - 1);  // conflict-free
    else w = (a >> 8) & (WORDS - 1);
    if (MODE == 0 || MODE == 2) atomicAdd((float*)&img[w], 1.0f);
    if (MODE == 1 || MODE == 3) atomicAdd(&img[w], 1u);
    if (MODE == 4) { float v = __uint_as_float(img[w]); img[w] = __float_as_uint(v + 1.0f); }
    if (MODE == 5) atomicAdd((unsigned long long*)&img[w & ~1u], 1ull);
    if (MODE == 6) { float2* p = (float2*)&img[w & ~1u]; float2 v = *p; v.x += 1.f; v.y += 1.f; *p = v; }
  }
  __syncthreads();
  uint32_t s = 0;
  for (int e = threadIdx.x; e < WORDS; e += 512) s += img[e];
  if (s == 0xdeadbeefu) out[0] = 1.0f;
}

int main() {
  float* out; CHK(hipMalloc(&out, 64));
  hipEvent_t a, b; CHK(hipEventCreate(&a)); CHK(hipEventCreate(&b));
  const int nb = 2048;
  const char* names[] = {"f32 atomic random", "u32 atomic random", "f32 atomic lane-linear",
                         "u32 atomic lane-linear", "f32 load+store random", "u64 atomic random",
                         "float2 load+store random"};
  auto run = [&](int m, auto launch) {
    float best = 1e9;
    for (int rep = 0; rep < 4; ++rep) {
      CHK(hipEventRecord(a)); launch(); CHK(hipGetLastError()); CHK(hipEventRecord(b));
      CHK(hipEventSynchronize(b)); float ms; CHK(hipEventElapsedTime(&ms, a, b)); if (ms < best) best = ms;
    }
    double ops = (double)nb * 512 * ITERS;
    printf("%-28s %8.1f us  %7.1f G lane-ops/s  %6.2f per CU-clock\n", names[m], best * 1e3,
           ops / (best * 1e-3) / 1e9, ops / (best * 1e-3) / (256 * 2.4e9));
  };
  run(0, [&] { k_lds<0><<<nb, 512>>>(out); });
  run(1, [&] { k_lds<1><<<nb, 512>>>(out); });
  run(2, [&] { k_lds<2><<<nb, 512>>>(out); });
  run(3, [&] { k_lds<3><<<nb, 512>>>(out); });
  run(4, [&] { k_lds<4><<<nb, 512>>>(out); });
  run(5, [&] { k_lds<5><<<nb, 512>>>(out); });
  run(6, [&] { k_lds<6><<<nb, 512>>>(out); });
  return 0;
}
