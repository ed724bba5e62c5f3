// vit_depuncture.hip -- de-puncturing (Sec. IV-E of the paper): expand a
// punctured soft-input stream into beta values per trellis stage, with a zero
// LLR (no information) in every punctured slot, so that the rate-1/beta
// decoder runs on it unchanged.  One thread per output stage; the received
// index of a kept slot is (t / period) * kept_per_period + the number of kept
// slots before it in the pattern.  Bandwidth-bound.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vit_internal.h"

namespace vit {
namespace {

template <typename T>
__global__ __launch_bounds__(256) void depuncture_kernel(const T *__restrict__ in, T *__restrict__ out,
                                                         int64_t stages, uint64_t mask, int32_t period,
                                                         int32_t beta, int32_t kept_per_period) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < stages; t += stride) {
    const int64_t q = t / period;
    const int p = (int)(t - q * period);
    for (int b = 0; b < beta; ++b) {
      const int pos = p * beta + b;
      T v = (T)0;
      if ((mask >> pos) & 1u) {
        const int before = __popcll(mask & ((1ull << pos) - 1ull));
        v = in[q * kept_per_period + before];
      }
      out[t * beta + b] = v;
    }
  }
}

}  // namespace

hipError_t launch_depuncture(const void *in, int llr_type, uint64_t mask, int32_t period, int32_t beta,
                             int32_t kept_per_period, int64_t stages, void *out, hipStream_t stream) {
  if (stages == 0) return hipSuccess;
  int64_t grid = (stages + 255) / 256;
  if (grid > 65536) grid = 65536;
  if (llr_type == VIT_LLR_F32)
    hipLaunchKernelGGL(depuncture_kernel<float>, dim3((unsigned)grid), dim3(256), 0, stream, (const float *)in,
                       (float *)out, stages, mask, period, beta, kept_per_period);
  else
    hipLaunchKernelGGL(depuncture_kernel<int8_t>, dim3((unsigned)grid), dim3(256), 0, stream, (const int8_t *)in,
                       (int8_t *)out, stages, mask, period, beta, kept_per_period);
  return hipGetLastError();
}

}  // namespace vit
