// vit_kernels16_k4.hip -- 16-bit modulo-metric kernel instances (stream and batch) for k = 4.
#include "vit_decoder16.h"

namespace vit {
void *pick_kernel16_k4(int beta, int in, bool batch) { return pick_kernel16_k<4>(beta, in, batch); }
}  // namespace vit
