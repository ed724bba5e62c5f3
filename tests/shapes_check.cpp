// Host-only check of the batch and serving launch rules in vit_shapes.h:
// default overlaps and the grid of a batch kernel (one workgroup per
// waves-per-workgroup items, or at most the occupancy grid for long blocks or
// low occupancy).  Prints "OK" and exits 0 when every check holds.
#include <stdio.h>

#include "vit_shapes.h"

static int failures = 0;
#define CHECK(cond)                                  \
  do {                                               \
    if (!(cond)) {                                   \
      printf("FAIL line %d: %s\n", __LINE__, #cond); \
      ++failures;                                    \
    }                                                \
  } while (0)

int main() {
  using vit::batch_grid;
  using vit::default_overlap;
  CHECK(default_overlap(3) == 15 && default_overlap(7) == 35);
  CHECK(default_overlap(8) == 56 && default_overlap(9) == 64);
  const int ncu = 256;
  // short blocks, many workgroups per CU: one workgroup per wpb items, at least 1
  CHECK(batch_grid(1000, 1, 547, 32u * ncu, ncu) == 1000);
  CHECK(batch_grid(1001, 2, 547, 16u * ncu, ncu) == 501);
  CHECK(batch_grid(0, 2, 547, 16u * ncu, ncu) == 1);
  CHECK(batch_grid(100000, 1, 999, 32u * ncu, ncu) == 100000);  // not capped below 1000 stages
  // blocks of 1000 stages or more: capped at the occupancy grid
  CHECK(batch_grid(100000, 1, 1000, 32u * ncu, ncu) == 32u * ncu);
  CHECK(batch_grid(100, 1, 1059, 32u * ncu, ncu) == 100);  // fewer items than the cap
  // 4 or fewer workgroups per CU: capped as well
  CHECK(batch_grid(100000, 2, 320, 4u * ncu, ncu) == 4u * ncu);
  CHECK(batch_grid(100000, 2, 320, 5u * ncu, ncu) == 50000);
  if (failures) return 1;
  printf("OK\n");
  return 0;
}
