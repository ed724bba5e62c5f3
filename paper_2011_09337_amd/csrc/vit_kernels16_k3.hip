// vit_kernels16_k3.hip -- 16-bit modulo-metric kernel instances (stream and batch) for k = 3.
#include "vit_decoder16.h"

namespace vit {
void *pick_kernel16_k3(int beta, int in, bool batch) { return pick_kernel16_k<3>(beta, in, batch); }
}  // namespace vit
