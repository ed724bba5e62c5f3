// vit_kernels_sub_k8.hip -- stream kernel instances with the subframe traceback, k = 8.
#include "vit_decoder.h"

namespace vit {
KernelFn pick_kernel_sub_k8(int beta, bool stdc, int in) { return pick_kernel_k<8, true>(beta, stdc, in); }
}  // namespace vit
