// vit_kernels_k5.hip -- kernel instances (stream and batch) for constraint length k = 5.
#include "vit_decoder.h"

namespace vit {
KernelFn pick_kernel_k5(int beta, bool stdc, int in) { return pick_kernel_k<5, false>(beta, stdc, in); }
BatchKernelFn pick_batch_kernel_k5(int beta, bool stdc, int in) { return pick_batch_kernel_k<5>(beta, stdc, in); }
}  // namespace vit
