// vit_kernels_sub_k5.hip -- stream kernel instances with the subframe traceback, k = 5.
#include "vit_decoder.h"

namespace vit {
KernelFn pick_kernel_sub_k5(int beta, bool stdc, int in) { return pick_kernel_k<5, true>(beta, stdc, in); }
}  // namespace vit
