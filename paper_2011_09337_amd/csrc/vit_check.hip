// vit_check.hip -- finiteness pre-pass over FP32 LLRs (vit_opts.check_finite).
// Bandwidth-bound: 16-byte loads where the buffer is 16-byte aligned; a lane
// that sees a NaN or an infinity sets one flag word with a vector atomic.
#include "vit_check.h"

#include <mutex>

namespace vit {
namespace {

__device__ __forceinline__ bool bad(float x) { return !__builtin_isfinite(x); }

__global__ __launch_bounds__(256) void clear_flag_kernel(uint32_t *flag) { *flag = 0u; }

__global__ __launch_bounds__(256) void nonfinite_kernel(const float *__restrict__ llr, int64_t count, int64_t nvec,
                                                        uint32_t *flag) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool any = false;
  for (int64_t i = tid; i < nvec; i += stride) {
    const float4 f = reinterpret_cast<const float4 *>(llr)[i];
    any = any || bad(f.x) || bad(f.y) || bad(f.z) || bad(f.w);
  }
  for (int64_t i = nvec * 4 + tid; i < count; i += stride) any = any || bad(llr[i]);
  if (any) atomicOr(flag, 1u);
}

constexpr int kMaxDevices = 64;
std::mutex g_mu;
uint32_t *g_flag[kMaxDevices];  // device flag word per device, allocated on first use
uint32_t *g_host;               // pinned host copy

}  // namespace

hipError_t check_finite_f32(const float *llr, int64_t count, hipStream_t stream, int *nonfinite) {
  *nonfinite = 0;
  if (count == 0) return hipSuccess;
  std::lock_guard<std::mutex> lock(g_mu);
  int dev = 0, ncu = 256;
  hipError_t err = hipGetDevice(&dev);
  if (err != hipSuccess) return err;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  if (!g_flag[dev]) {
    err = hipMalloc(reinterpret_cast<void **>(&g_flag[dev]), 256);
    if (err != hipSuccess) return err;
  }
  if (!g_host) {
    err = hipHostMalloc(reinterpret_cast<void **>(&g_host), 256, hipHostMallocDefault);
    if (err != hipSuccess) return err;
  }
  err = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (err != hipSuccess) return err;
  const int64_t nvec = (((uintptr_t)llr) & 15u) == 0 ? count / 4 : 0;
  const int64_t work = nvec + (count - nvec * 4);
  int64_t grid = (work + 255) / 256;
  const int64_t cap = (int64_t)ncu * 8;
  if (grid > cap) grid = cap;
  if (grid < 1) grid = 1;
  // the flag is cleared by a kernel, not a memset, so the pass may sit in a captured graph
  hipLaunchKernelGGL(clear_flag_kernel, dim3(1), dim3(1), 0, stream, g_flag[dev]);
  hipLaunchKernelGGL(nonfinite_kernel, dim3((unsigned)grid), dim3(256), 0, stream, llr, count, nvec, g_flag[dev]);
  err = hipGetLastError();
  if (err != hipSuccess) return err;
  err = hipMemcpyAsync(g_host, g_flag[dev], sizeof(uint32_t), hipMemcpyDeviceToHost, stream);
  if (err != hipSuccess) return err;
  err = hipStreamSynchronize(stream);
  if (err != hipSuccess) return err;
  *nonfinite = *g_host != 0u;
  return hipSuccess;
}

}  // namespace vit
