// vit_kernels_k6.hip -- kernel instances (stream and batch) for constraint length k = 6.
#include "vit_decoder.h"

namespace vit {
KernelFn pick_kernel_k6(int beta, bool stdc, int in) { return pick_kernel_k<6, false>(beta, stdc, in); }
BatchKernelFn pick_batch_kernel_k6(int beta, bool stdc, int in) { return pick_batch_kernel_k<6>(beta, stdc, in); }
}  // namespace vit
