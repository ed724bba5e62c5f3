// vit_kernels_k5.hip -- kernel instances (stream and batch) for constraint length k = 5.
#include "vit_decoder.h"

namespace vit {
KernelFn pick_kernel_k5(int beta, bool stdc, bool i8) { return pick_kernel_k<5, false>(beta, stdc, i8); }
BatchKernelFn pick_batch_kernel_k5(int beta, bool stdc, bool i8) { return pick_batch_kernel_k<5>(beta, stdc, i8); }
}  // namespace vit
