// vit_kernels_k9.hip -- kernel instances (stream and batch) for constraint length k = 9.
#include "vit_decoder.h"

namespace vit {
KernelFn pick_kernel_k9(int beta, bool stdc, int in) { return pick_kernel_k<9, false>(beta, stdc, in); }
BatchKernelFn pick_batch_kernel_k9(int beta, bool stdc, int in) { return pick_batch_kernel_k<9>(beta, stdc, in); }
}  // namespace vit
