// vit_kernels_k3.hip -- kernel instances (stream and batch) for constraint length k = 3.
#include "vit_decoder.h"

namespace vit {
KernelFn pick_kernel_k3(int beta, bool stdc, bool i8) { return pick_kernel_k<3, false>(beta, stdc, i8); }
BatchKernelFn pick_batch_kernel_k3(int beta, bool stdc, bool i8) { return pick_batch_kernel_k<3>(beta, stdc, i8); }
}  // namespace vit
