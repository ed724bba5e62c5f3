// vit_kernels_sub_k6.hip -- stream kernel instances with the subframe traceback, k = 6.
#include "vit_decoder.h"

namespace vit {
KernelFn pick_kernel_sub_k6(int beta, bool stdc, int in) { return pick_kernel_k<6, true>(beta, stdc, in); }
}  // namespace vit
