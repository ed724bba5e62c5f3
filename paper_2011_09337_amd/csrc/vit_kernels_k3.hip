// vit_kernels_k3.hip -- kernel instances (stream and batch) for constraint length k = 3.
#include "vit_decoder.h"

namespace vit {
KernelFn pick_kernel_k3(int beta, bool stdc, int in) { return pick_kernel_k<3, false>(beta, stdc, in); }
BatchKernelFn pick_batch_kernel_k3(int beta, bool stdc, int in) { return pick_batch_kernel_k<3>(beta, stdc, in); }
}  // namespace vit
