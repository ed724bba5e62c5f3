// vit_quantize.hip -- int8 quantisation of soft inputs:
//   q = clamp(round_half_even(llr * scale), -127, 127).
// The product is rounded once to fp32 (v_mul_f32, round to nearest even),
// then to the nearest integer with ties to even (v_rndne_f32), then clamped;
// -128 is never produced, so negating a quantised LLR cannot overflow.
// Bandwidth-bound: each thread converts 16 values with 16-byte loads/stores
// when both buffers are 16-byte aligned, and the remainder one by one.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vit_internal.h"

namespace vit {
namespace {

__device__ __forceinline__ int8_t q8(float x, float scale) {
  float y = __builtin_rintf(x * scale);  // rint rounds to nearest even in the default mode
  y = __builtin_fminf(__builtin_fmaxf(y, -127.0f), 127.0f);
  return (int8_t)(int)y;
}

// Vectors [0, nvec) of 16 values, then scalars [nvec*16, count).
__global__ __launch_bounds__(256) void quantize_kernel(const float *__restrict__ llr, int64_t count, int64_t nvec,
                                                       float scale, int8_t *__restrict__ q) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t i = tid; i < nvec; i += stride) {
    const float4 *src = reinterpret_cast<const float4 *>(llr) + i * 4;
    uint32_t w[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float4 f = src[j];
      w[j] = (uint32_t)(uint8_t)q8(f.x, scale) | ((uint32_t)(uint8_t)q8(f.y, scale) << 8) |
             ((uint32_t)(uint8_t)q8(f.z, scale) << 16) | ((uint32_t)(uint8_t)q8(f.w, scale) << 24);
    }
    reinterpret_cast<uint4 *>(q)[i] = make_uint4(w[0], w[1], w[2], w[3]);
  }
  for (int64_t i = nvec * 16 + tid; i < count; i += stride) q[i] = q8(llr[i], scale);
}

}  // namespace

hipError_t launch_quantize(const float *llr, int64_t count, float scale, int8_t *q, hipStream_t stream) {
  if (count == 0) return hipSuccess;
  int dev = 0, ncu = 256;
  hipError_t err = hipGetDevice(&dev);
  if (err != hipSuccess) return err;
  err = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (err != hipSuccess) return err;
  const bool aligned = (((uintptr_t)llr | (uintptr_t)q) & 15u) == 0;
  const int64_t nvec = aligned ? count / 16 : 0;
  const int64_t work = nvec + (count - nvec * 16);
  int64_t grid = (work + 255) / 256;
  const int64_t cap = (int64_t)ncu * 8;
  if (grid > cap) grid = cap;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(quantize_kernel, dim3((unsigned)grid), dim3(256), 0, stream, llr, count, nvec, scale, q);
  return hipGetLastError();
}

}  // namespace vit
