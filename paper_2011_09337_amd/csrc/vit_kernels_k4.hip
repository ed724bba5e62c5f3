// vit_kernels_k4.hip -- kernel instances (stream and batch) for constraint length k = 4.
#include "vit_decoder.h"

namespace vit {
KernelFn pick_kernel_k4(int beta, bool stdc, int in) { return pick_kernel_k<4, false>(beta, stdc, in); }
BatchKernelFn pick_batch_kernel_k4(int beta, bool stdc, int in) { return pick_batch_kernel_k<4>(beta, stdc, in); }
}  // namespace vit
