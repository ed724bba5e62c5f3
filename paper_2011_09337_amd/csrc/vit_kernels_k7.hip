// vit_kernels_k7.hip -- kernel instances (stream and batch) for constraint length k = 7.
#include "vit_decoder.h"

namespace vit {
KernelFn pick_kernel_k7(int beta, bool stdc, int in) { return pick_kernel_k<7, false>(beta, stdc, in); }
BatchKernelFn pick_batch_kernel_k7(int beta, bool stdc, int in) { return pick_batch_kernel_k<7>(beta, stdc, in); }
}  // namespace vit
