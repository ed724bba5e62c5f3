// vit_kernels16_k7.hip -- 16-bit modulo-metric kernel instances (stream and batch) for k = 7.
#include "vit_decoder16.h"

namespace vit {
void *pick_kernel16_k7(int beta, int in, bool batch) { return pick_kernel16_k<7>(beta, in, batch); }
}  // namespace vit
