// vit_shapes.h -- default block shapes and launch grids of the batch and
// serving paths.
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

// Workgroups for one batch decode kernel over `count` work items, `wpb` waves
// per workgroup, blocks of at most `max_block_stages` stages.  The kernel's
// waves stride over the items, so any grid is correct.  Normally one workgroup
// per wpb items, which the dispatcher refills on a CU as workgroups end; for
// blocks of 1000 stages or more, or when at most 4 workgroups fit on a CU
// (occ_grid <= 4 * num_cu), at most occ_grid (one wave per resident slot)
// persistent waves, which keep fewer long tails.  Same rule as the stream
// kernel's launch.
inline unsigned batch_grid(int64_t count, int wpb, int64_t max_block_stages, unsigned occ_grid, int num_cu) {
  int64_t g = (count + wpb - 1) / wpb;
  if (g < 1) g = 1;
  const bool persistent = max_block_stages >= 1000 || occ_grid <= 4u * (unsigned)num_cu;
  if (persistent && g > (int64_t)occ_grid) g = occ_grid;
  return (unsigned)g;
}

}  // namespace vit
