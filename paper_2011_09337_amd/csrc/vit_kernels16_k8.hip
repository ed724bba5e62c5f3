// vit_kernels16_k8.hip -- 16-bit modulo-metric kernel instances (stream and batch) for k = 8.
#include "vit_decoder16.h"

namespace vit {
void *pick_kernel16_k8(int beta, int in, bool batch) { return pick_kernel16_k<8>(beta, in, batch); }
}  // namespace vit
