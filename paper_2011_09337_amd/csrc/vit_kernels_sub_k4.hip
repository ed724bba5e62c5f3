// vit_kernels_sub_k4.hip -- stream kernel instances with the subframe traceback, k = 4.
#include "vit_decoder.h"

namespace vit {
KernelFn pick_kernel_sub_k4(int beta, bool stdc, int in) { return pick_kernel_k<4, true>(beta, stdc, in); }
}  // namespace vit
