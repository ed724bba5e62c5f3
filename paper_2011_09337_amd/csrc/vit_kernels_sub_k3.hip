// vit_kernels_sub_k3.hip -- stream kernel instances with the subframe traceback, k = 3.
#include "vit_decoder.h"

namespace vit {
KernelFn pick_kernel_sub_k3(int beta, bool stdc, bool i8) { return pick_kernel_k<3, true>(beta, stdc, i8); }
}  // namespace vit
