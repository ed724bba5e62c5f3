// vit_kernels16_k6.hip -- 16-bit modulo-metric kernel instances (stream and batch) for k = 6.
#include "vit_decoder16.h"

namespace vit {
void *pick_kernel16_k6(int beta, int in, bool batch) { return pick_kernel16_k<6>(beta, in, batch); }
}  // namespace vit
