// vit_shapes.h -- default block shapes of the batch and serving paths.
#pragma once

#include <stdint.h>

namespace vit {

// Total overlap v (v1 = floor(v/2) on the left, the rest on the right) used
// when the caller gives no shape: 5k up to k = 7; 8(k-1) from k = 8 on.  The
// longer codes need the longer traceback: measured on 2^24-bit streams at
// BER 1e-4, K=9 r1/2 int8 blocks of 256 bits sit 0.148 dB from maximum
// likelihood at v = 45 and 0.084 / 0.059 dB at v = 60 / 72; K=7 r1/2 int8 at
// v = 35 sits 0.041 dB from it.
inline int32_t default_overlap(int32_t k) { return k <= 7 ? 5 * k : 8 * (k - 1); }

}  // namespace vit
