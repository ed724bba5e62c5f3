// vit_kernels16_k9.hip -- 16-bit modulo-metric kernel instances (stream and batch) for k = 9.
#include "vit_decoder16.h"

namespace vit {
void *pick_kernel16_k9(int beta, int in, bool batch) { return pick_kernel16_k<9>(beta, in, batch); }
}  // namespace vit
