// vit_kernels_k8.hip -- kernel instances (stream and batch) for constraint length k = 8.
#include "vit_decoder.h"

namespace vit {
KernelFn pick_kernel_k8(int beta, bool stdc, int in) { return pick_kernel_k<8, false>(beta, stdc, in); }
BatchKernelFn pick_batch_kernel_k8(int beta, bool stdc, int in) { return pick_batch_kernel_k<8>(beta, stdc, in); }
}  // namespace vit
