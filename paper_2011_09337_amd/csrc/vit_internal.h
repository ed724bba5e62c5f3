// vit_internal.h -- shared between the host API (vit_api.cpp) and the HIP
// kernels (vit_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vit.h"

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
  int32_t llr_type;      // VIT_LLR_F32, VIT_LLR_I8 or VIT_LLR_HARD
  int32_t max_block_stages;
  int32_t sub_bits;      // > 0: parallel traceback in subframes of this many core bits; 0: one per block
  int32_t sub_overlap;   // inner overlap of a subframe, in stages
  int32_t sub_start;     // VIT_SUBFRAME_STORED or VIT_SUBFRAME_RANDOM
  uint64_t sub_seed;     // SplitMix64 seed of the random start rule
  int32_t metric_bits;   // integer inputs: 16 (modulo 2^16 metrics), 32 (exact integers held in fp32), 0 = 32
                         // where its bound and survivor storage allow, else 16
};

// Path metrics of the integer kernels (int8 and hard-decision inputs).
constexpr int kMetricAuto = 0;
constexpr int kMetric16 = 16;
constexpr int kMetric32 = 32;

// One work item of a batched decode: one block of one frame.
struct WorkItem {
  int64_t llr_off;       // byte offset of the frame's first LLR in the batch buffer
  int64_t out_off;       // byte offset of the frame's first decoded byte
  int32_t s, e;          // frame-local stage window
  int32_t cs, ce;        // frame-local core bits
  int32_t flags;         // bit 0: window starts at stage 0; bit 1: ends at the last stage of a terminated frame
  int32_t cost;          // stages x states / 64 (for sorting)
};

// Workspace header of a batched decode (device, int32 words): for code c,
// [kMaxCodes + c] = number of items, [2*kMaxCodes + c] = offset of its first
// item in the item array; words [0, kMaxCodes) are reserved (zero).
constexpr int kMaxCodes = 8;
constexpr size_t kHeaderBytes = 256;

// Kernel arguments of a batched decode for one code.
struct BatchArgs {
  const void *llr;           // device, the batch's LLR buffer
  uint8_t *out;              // device, the batch's output buffer
  int32_t *header;           // device, workspace header
  const WorkItem *items;     // device, all work items (each code's run is cost-descending)
  int32_t code_index;
  uint32_t gen[4];
};

// Survivor (decision) storage of one block in LDS, in bytes, for a kernel
// instance: groups of 32 stages x states/8 bytes, rounded up to whole bodies
// of the unrolled loop.  0 if (k, beta) has no kernel instance.
int64_t lds_bytes_per_block(int k, int beta, int64_t max_block_stages);
// The same for a wave of the 16-bit metric kernels, which decodes two blocks
// at once: one dword per slot per body of up to 16 stages.
int64_t lds16_bytes_per_wave(int k, int beta, int64_t max_block_stages);
// Integer metrics exact in fp32: (stages of a block) x 128 x beta < 2^24.
bool fp32_integer_exact(int beta, int64_t max_block_stages);

// Launch the blocked decoder on `stream`.  Returns hipSuccess or the HIP error.
// *unsupported is set (and hipSuccess returned) if no kernel instance exists
// or the LDS need exceeds the device limit.
hipError_t launch_blocked(const DecodeArgs &a, hipStream_t stream, int *unsupported,
                          const char **why);

// Kernel instance and launch shape of a batched decode for one code.
struct BatchLaunch {
  const void *fn;            // __global__ function
  unsigned grid, block;      // workgroups, threads per workgroup
  size_t lds;                // dynamic LDS bytes per workgroup
  int lds_words_per_wave;
  int items_per_wave;        // work items a wave takes at once (2 for the 16-bit metric kernels)
  int metric_bits;           // 16 or 32 for integer inputs, 0 for FP32
};
// Fill *bl for a code (k, beta, generators, input kind, metric choice as
// DecodeArgs::metric_bits) decoding blocks of at most max_block_stages
// stages with `wpb` waves per workgroup.  Returns hipSuccess; sets
// *unsupported when the shape is not available.
hipError_t plan_batch_launch(int k, int beta, const uint32_t *gen, int in, int metric_bits, int64_t max_block_stages,
                             int wpb, BatchLaunch *bl, int *unsupported, const char **why);
// Workgroups of one batch kernel launch over `count` work items (the grid rule
// of vit_shapes.h applied to the waves' units of work).
unsigned batch_launch_grid(const BatchLaunch &bl, int64_t count, int64_t max_block_stages, int num_cu);

// Error reporting shared by the C ABI translation units (thread-local message).
void api_clear_error();
int api_fail(int status, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int api_fail_hip(hipError_t e, const char *what);
int api_check_code(const vit_code *c);
// The integer kernels' limits that need no device: VIT_EUNSUPPORTED (with the
// message set) when no integer kernel can take blocks of max_block_stages
// stages under the metric choice, VIT_OK otherwise (and for FP32 inputs).
int integer_shape_precheck(int k, int beta, int llr_type, int metric_bits, int64_t max_block_stages, bool subframes);

// A byte range to copy on the device (either side may be pinned host memory
// mapped for the device).  32 bytes, the layout the copy kernel reads.
struct CopyRange {
  const uint8_t *src;
  uint8_t *dst;
  int64_t bytes;
  int64_t pad;
};
// Copy `count` ranges listed in device memory (vit_copy.hip).
hipError_t launch_copy_list(const CopyRange *ranges, int32_t count, hipStream_t stream);

// Launch the de-puncturer (vit_depuncture.hip): pattern bits mask[p*beta + b],
// kept_per_period of them set.
hipError_t launch_depuncture(const void *in, int llr_type, uint64_t mask, int32_t period, int32_t beta,
                             int32_t kept_per_period, int64_t stages, void *out, hipStream_t stream);

// Launch the int8 quantiser (vit_quantize.hip) on `stream`.
hipError_t launch_quantize(const float *llr, int64_t count, float scale, int8_t *q, hipStream_t stream);

}  // namespace vit
