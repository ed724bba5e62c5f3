// vit_check.h -- the optional finiteness pre-pass over FP32 LLRs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vit {

// Scan count FP32 values at llr (device) on `stream` and wait for the scan:
// *nonfinite = 1 if any is NaN or infinite, else 0.  Calls are serialised
// (one flag word per device).
hipError_t check_finite_f32(const float *llr, int64_t count, hipStream_t stream, int *nonfinite);

}  // namespace vit
