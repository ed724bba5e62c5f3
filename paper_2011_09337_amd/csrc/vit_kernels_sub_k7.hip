// vit_kernels_sub_k7.hip -- stream kernel instances with the subframe traceback, k = 7.
#include "vit_decoder.h"

namespace vit {
KernelFn pick_kernel_sub_k7(int beta, bool stdc, int in) { return pick_kernel_k<7, true>(beta, stdc, in); }
}  // namespace vit
