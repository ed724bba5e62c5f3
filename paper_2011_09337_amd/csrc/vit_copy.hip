// vit_copy.hip -- copies of a list of byte ranges, used by the serving loop
// to move its work list and the LLRs of newly admitted frames from pinned
// host memory into the device in one launch per iteration, however many
// frames it holds (the decode kernels write the decoded bytes back into the
// host region themselves).  The range list itself may sit in device memory or
// in mapped pinned host memory.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vit_internal.h"

namespace vit {
namespace {

// One workgroup per range (grid-strided): 16-byte words when source,
// destination and length allow, bytes otherwise.  Each thread has four words
// in flight before it stores, since a read across PCIe takes microseconds.
__global__ __launch_bounds__(256) void copy_list_kernel(const CopyRange *__restrict__ r, int32_t count) {
  for (int32_t i = blockIdx.x; i < count; i += gridDim.x) {
    const uint8_t *src = r[i].src;
    uint8_t *dst = r[i].dst;
    const int64_t bytes = r[i].bytes;
    int64_t done = 0;
    if ((((uintptr_t)src | (uintptr_t)dst) & 15u) == 0) {
      const int64_t nw = bytes >> 4;
      const int64_t bd = blockDim.x;
      const uint4 *s4 = reinterpret_cast<const uint4 *>(src);
      uint4 *d4 = reinterpret_cast<uint4 *>(dst);
      int64_t j = threadIdx.x;
      for (; j + 3 * bd < nw; j += 4 * bd) {
        const uint4 a = s4[j], b = s4[j + bd], c = s4[j + 2 * bd], d = s4[j + 3 * bd];
        d4[j] = a;
        d4[j + bd] = b;
        d4[j + 2 * bd] = c;
        d4[j + 3 * bd] = d;
      }
      for (; j < nw; j += bd) d4[j] = s4[j];
      done = nw << 4;
    }
    for (int64_t j = done + threadIdx.x; j < bytes; j += blockDim.x) dst[j] = src[j];
  }
}

}  // namespace

hipError_t launch_copy_list(const CopyRange *ranges, int32_t count, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  const int grid = count < 2048 ? count : 2048;
  hipLaunchKernelGGL(copy_list_kernel, dim3(grid), dim3(256), 0, stream, ranges, count);
  return hipGetLastError();
}

}  // namespace vit
