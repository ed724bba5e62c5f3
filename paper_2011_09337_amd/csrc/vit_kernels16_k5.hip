// vit_kernels16_k5.hip -- 16-bit modulo-metric kernel instances (stream and batch) for k = 5.
#include "vit_decoder16.h"

namespace vit {
void *pick_kernel16_k5(int beta, int in, bool batch) { return pick_kernel16_k<5>(beta, in, batch); }
}  // namespace vit
