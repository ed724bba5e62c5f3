// vit_kernels_sub_k3.hip -- stream kernel instances with the subframe traceback, k = 3.
#include "vit_decoder.h"

namespace vit {
KernelFn pick_kernel_sub_k3(int beta, bool stdc, int in) { return pick_kernel_k<3, true>(beta, stdc, in); }
}  // namespace vit
