// vit_kernels_k9.hip -- kernel instances (stream and batch) for constraint length k = 9.
#include "vit_decoder.h"

namespace vit {
KernelFn pick_kernel_k9(int beta, bool stdc, bool i8) { return pick_kernel_k<9, false>(beta, stdc, i8); }
BatchKernelFn pick_batch_kernel_k9(int beta, bool stdc, bool i8) { return pick_batch_kernel_k<9>(beta, stdc, i8); }
}  // namespace vit
