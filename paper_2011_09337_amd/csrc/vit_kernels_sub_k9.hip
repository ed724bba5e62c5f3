// vit_kernels_sub_k9.hip -- stream kernel instances with the subframe traceback, k = 9.
#include "vit_decoder.h"

namespace vit {
KernelFn pick_kernel_sub_k9(int beta, bool stdc, int in) { return pick_kernel_k<9, true>(beta, stdc, in); }
}  // namespace vit
