// vit_kernels_k4.hip -- kernel instances (stream and batch) for constraint length k = 4.
#include "vit_decoder.h"

namespace vit {
KernelFn pick_kernel_k4(int beta, bool stdc, bool i8) { return pick_kernel_k<4, false>(beta, stdc, i8); }
BatchKernelFn pick_batch_kernel_k4(int beta, bool stdc, bool i8) { return pick_batch_kernel_k<4>(beta, stdc, i8); }
}  // namespace vit
