// vit_internal.h -- shared between the host API (vit_api.cpp) and the HIP
// kernels (vit_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vit {

// Arguments of one blocked decode, resolved by the host (geometry already
// validated; L > 0 and a multiple of 8 or the single full-frame block).
struct DecodeArgs {
  const void *llr;       // device, N*beta LLRs (float or int8)
  uint8_t *out;          // device, ceil(n/8) bytes
  int64_t n;             // information bits
  int64_t N;             // trellis stages in the stream
  int64_t L;             // core bits per block
  int64_t v1, v2;        // left / right overlap
  int64_t nblocks;       // ceil(n / L)
  uint32_t gen[4];
  int32_t k, beta;
  int32_t terminated;
  int32_t llr_type;      // VIT_LLR_F32 or VIT_LLR_I8
  int32_t max_block_stages;
};

// Survivor (decision) storage of one block in LDS, in bytes, for a kernel
// instance: groups of 32 stages x states/8 bytes, rounded up to whole bodies
// of the unrolled loop.  0 if (k, beta) has no kernel instance.
int64_t lds_bytes_per_block(int k, int beta, int64_t max_block_stages);

// Launch the blocked decoder on `stream`.  Returns hipSuccess or the HIP error.
// *unsupported is set (and hipSuccess returned) if no kernel instance exists
// or the LDS need exceeds the device limit.
hipError_t launch_blocked(const DecodeArgs &a, hipStream_t stream, int *unsupported,
                          const char **why);

// Launch the int8 quantiser (vit_quantize.hip) on `stream`.
hipError_t launch_quantize(const float *llr, int64_t count, float scale, int8_t *q, hipStream_t stream);

}  // namespace vit
