// Matrix-core rate probe: the sustained MFMA rate of the device, measured
// beside the datasheet peak against which the MLP kernel's rate is stated.
// Kept out of the training kernels' source.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "romap_device.h"

typedef float rmp_floatx4 __attribute__((ext_vector_type(4)));
typedef float rmp_floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 rmp_bf16x8 __attribute__((ext_vector_type(8)));

// Each wave runs `iters` rounds of CH independent accumulator chains with no
// memory traffic in the loop.  PREC 1: 32x32x16 BF16 (32768 flops per
// instruction; on gfx950 it sustains more than the 16x16x32 shape, whose
// dependent-issue latency needs twice the chains); PREC 0: 16x16x4 FP32
// (2048 flops).
template <int PREC>
__global__ __launch_bounds__(256) void k_mfma_rate(int iters, float* out) {
  const int lane = threadIdx.x & 63;
  float t = 0.0f;
  if constexpr (PREC == 1) {
    constexpr int CH = 2;
    rmp_floatx16 acc[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[c][r] = 0.0f;
    rmp_bf16x8 x;
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = (__bf16)(1.0f / 1024.0f * (float)((lane + k) & 7));
    for (int it = 0; it < iters; ++it) {
#pragma unroll
      for (int c = 0; c < CH; ++c) acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x, x, acc[c], 0, 0, 0);
    }
#pragma unroll
    for (int c = 0; c < CH; ++c) t += acc[c][0] + acc[c][15];
  } else {
    constexpr int CH = 16;
    rmp_floatx4 acc[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) acc[c] = rmp_floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    const float x = 1.0f / 1024.0f * (float)(lane & 7);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
      for (int c = 0; c < CH; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(x, x, acc[c], 0, 0, 0);
    }
#pragma unroll
    for (int c = 0; c < CH; ++c) t += acc[c][0] + acc[c][3];
  }
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = t;
}

// flops of one launch of `blocks` 4-wave workgroups running `iters` rounds
double rm_mfma_rate_flops(int prec, int blocks, int iters) {
  return prec == 1 ? (double)blocks * 4 * iters * 2 * 32768.0
                   : (double)blocks * 4 * iters * 16 * 2048.0;
}

hipError_t rm_launch_mfma_rate(int prec, int blocks, int iters, float* out, hipStream_t st) {
  if (prec == 1)
    k_mfma_rate<1><<<blocks, 256, 0, st>>>(iters, out);
  else
    k_mfma_rate<0><<<blocks, 256, 0, st>>>(iters, out);
  return hipGetLastError();
}
