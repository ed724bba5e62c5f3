// vit_batch_items.h -- work lists of batched decodes, shared by the plan path
// (vit_batch.cpp) and the allocation-free entry point (vit_batch_static.cpp).
// Not part of the public ABI.
#pragma once

#include <stdint.h>

#include <utility>

#include "vit.h"
#include "vit_internal.h"

namespace vit {

// Default block shape of a code: L = 256, the default overlap, one wave per
// workgroup.
vit_tuning default_tuning(const vit_code &c);
int check_tuning(const vit_tuning &t);
// codes (1..8, each valid) and a non-empty frame list.
int check_batch_args(const vit_code *codes, int32_t ncodes, const vit_frame *frames, int32_t nframes);
// Every frame against the buffers (code id, lengths, LLR and output ranges
// inside the buffers, output ranges disjoint).  outs: caller storage for
// nframes ranges (sorted in place).
int check_frames(const vit_code *codes, int32_t ncodes, const vit_frame *frames, int32_t nframes, int64_t llr_count,
                 int llr_type, int64_t out_bytes, std::pair<int64_t, int64_t> *outs);
// Work items of every frame under the given shapes (Sec. III per frame): the
// item count is returned; with items != NULL also the items, each code's run
// sorted by cost (longest first), the header's per-code counts and offsets,
// and max_stages[c].  tmp must hold the longest code run, hist
// max(L + v) + 2 counters.
int64_t build_items(const vit_code *codes, int32_t ncodes, const vit_frame *frames, int32_t nframes,
                    const vit_tuning *shape, int elem_bytes, WorkItem *items, int32_t *header, int64_t *max_stages,
                    WorkItem *tmp, int64_t *hist);
// Launch order of the codes' kernels: most work per bit (states x rate) first.
void batch_code_order(const vit_code *codes, int32_t ncodes, int *order);

}  // namespace vit
