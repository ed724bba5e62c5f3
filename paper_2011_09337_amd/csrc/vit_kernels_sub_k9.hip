// vit_kernels_sub_k9.hip -- stream kernel instances with the subframe traceback, k = 9.
#include "vit_decoder.h"

namespace vit {
KernelFn pick_kernel_sub_k9(int beta, bool stdc, bool i8) { return pick_kernel_k<9, true>(beta, stdc, i8); }
}  // namespace vit
