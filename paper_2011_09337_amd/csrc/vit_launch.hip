// vit_launch.hip -- host side of the blocked decoder: kernel selection,
// occupancy-based grid size, LDS sizing and launch.
#include "vit_decoder.h"
#include "vit_decoder16.h"
#include "vit_shapes.h"

namespace vit {
namespace {


KernelFn pick_kernel(int k, int beta, bool stdc, int in, bool sub) {
  switch (k) {
    case 3: return sub ? pick_kernel_sub_k3(beta, stdc, in) : pick_kernel_k3(beta, stdc, in);
    case 4: return sub ? pick_kernel_sub_k4(beta, stdc, in) : pick_kernel_k4(beta, stdc, in);
    case 5: return sub ? pick_kernel_sub_k5(beta, stdc, in) : pick_kernel_k5(beta, stdc, in);
    case 6: return sub ? pick_kernel_sub_k6(beta, stdc, in) : pick_kernel_k6(beta, stdc, in);
    case 7: return sub ? pick_kernel_sub_k7(beta, stdc, in) : pick_kernel_k7(beta, stdc, in);
    case 8: return sub ? pick_kernel_sub_k8(beta, stdc, in) : pick_kernel_k8(beta, stdc, in);
    case 9: return sub ? pick_kernel_sub_k9(beta, stdc, in) : pick_kernel_k9(beta, stdc, in);
  }
  return nullptr;
}

int body_len(int k) {
  const int P = k - 1;
  return P * (32 / P);
}

void *pick_kernel16(int k, int beta, int in, bool batch) {
  switch (k) {
    case 3: return pick_kernel16_k3(beta, in, batch);
    case 4: return pick_kernel16_k4(beta, in, batch);
    case 5: return pick_kernel16_k5(beta, in, batch);
    case 6: return pick_kernel16_k6(beta, in, batch);
    case 7: return pick_kernel16_k7(beta, in, batch);
    case 8: return pick_kernel16_k8(beta, in, batch);
    case 9: return pick_kernel16_k9(beta, in, batch);
  }
  return nullptr;
}

struct DeviceInfo {
  int dev = -1;
  int num_cu = 0;
  int max_lds = 0;
};
thread_local DeviceInfo t_dev;

}  // namespace

int64_t lds_bytes_per_block(int k, int beta, int64_t max_block_stages) {
  if (k < 3 || k > 9 || beta < 2 || beta > 4) return 0;
  const int64_t body = body_len(k);
  const int64_t regs = (k > 7) ? (1 << (k - 1)) / 64 : 1;
  const int64_t bodies = (max_block_stages + body - 1) / body;  // block + entry offset fill whole bodies
  return bodies * regs * 64 * 4;
}

int64_t lds16_bytes_per_wave(int k, int beta, int64_t max_block_stages) {
  if (k < 3 || k > 9 || beta < 2 || beta > 4) return 0;
  const int64_t body = dev16::body16(k - 1);
  const int64_t regs = (k > 7) ? (1 << (k - 1)) / 64 : 1;
  const int64_t bodies = (max_block_stages + body - 1) / body;
  return bodies * regs * 64 * 4;
}

bool fp32_integer_exact(int beta, int64_t max_block_stages) {
  return max_block_stages * 128 * beta < ((int64_t)1 << 24);
}

namespace {

hipError_t device_info() {
  int dev = 0;
  hipError_t err = hipGetDevice(&dev);
  if (err != hipSuccess) return err;
  if (t_dev.dev != dev) {
    err = hipDeviceGetAttribute(&t_dev.num_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (err != hipSuccess) return err;
    err = hipDeviceGetAttribute(&t_dev.max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (err != hipSuccess) return err;
    t_dev.dev = dev;
  }
  return hipSuccess;
}

// Resolve the integer metric width for a decode of blocks of at most
// max_block_stages stages: the 16-bit kernels where asked for, the
// exact-in-fp32 integer kernels where asked for or (auto) where their bound
// and their survivor storage allow, else (auto) the 16-bit kernels where two
// blocks' survivors fit a workgroup's LDS.  Auto prefers the 32-bit kernels
// because they measured faster on gfx950 (the 16-bit kernels hold two
// blocks' survivors per wave, which halves the waves the LDS admits).
// -1 = no kernel (why is set).
int resolve_metric(int k, int beta, int in, int metric_bits, int64_t max_block_stages, const char **why) {
  if (in == VIT_LLR_F32) return 0;
  const bool fits16 = lds16_bytes_per_wave(k, beta, max_block_stages) <= t_dev.max_lds;
  const bool fits32 = lds_bytes_per_block(k, beta, max_block_stages) <= t_dev.max_lds &&
                      fp32_integer_exact(beta, max_block_stages);
  if (metric_bits == kMetric16 || (metric_bits == kMetricAuto && !fits32 && fits16)) {
    if (!fits16) *why = "the 16-bit metric kernel's survivor storage for two blocks exceeds the per-workgroup LDS";
    return fits16 ? kMetric16 : -1;
  }
  if (!fits32) {
    *why = lds_bytes_per_block(k, beta, max_block_stages) > t_dev.max_lds
               ? "one block's survivor storage exceeds the per-workgroup LDS"
               : "int8 block too long for exact integers in fp32 (use 16-bit metrics)";
    return -1;
  }
  return kMetric32;
}

// The 16-bit metric stream kernel: one wave per pair of blocks.
hipError_t launch_blocked16(const DecodeArgs &a, hipStream_t stream, int *unsupported, const char **why) {
  void *fn = pick_kernel16(a.k, a.beta, a.llr_type, false);
  if (!fn) {
    *unsupported = 1;
    *why = "no 16-bit metric kernel instance for this (k, beta)";
    return hipSuccess;
  }
  const int64_t lds_wave = lds16_bytes_per_wave(a.k, a.beta, a.max_block_stages);
  int wpb = (2 * lds_wave <= t_dev.max_lds) ? 2 : 1;
  int occ = 0;
  hipError_t err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, 64 * wpb, (size_t)lds_wave * wpb);
  if (err != hipSuccess) return err;
  if (occ < 1) occ = 1;
  // same rule as the one-block-per-wave kernels (launch_blocked), in pairs
  const bool persistent = a.max_block_stages >= 1000 || occ <= 4;
  if (!persistent) wpb = 1;
  const size_t lds = (size_t)lds_wave * wpb;
  const int64_t npairs = (a.nblocks + 1) / 2;
  const int64_t need = (npairs + wpb - 1) / wpb;
  int64_t grid = need;
  if (persistent) {
    grid = (int64_t)occ * t_dev.num_cu;
    if (grid >= need) grid = need;
    else grid = grid / 8 * 8;
  }
  if (grid < 1) grid = 1;
  if (lds > 65536) {
    err = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (err != hipSuccess) return err;
  }
  DecodeArgs args = a;
  int words = (int)(lds_wave / 4);
  void *kargs[] = {&args, &words};
  err = hipLaunchKernel(fn, dim3((unsigned)grid), dim3(64 * wpb), kargs, lds, stream);
  if (err != hipSuccess) return err;
  return hipGetLastError();
}

}  // namespace

hipError_t launch_blocked(const DecodeArgs &a, hipStream_t stream, int *unsupported, const char **why) {
  *unsupported = 0;
  {
    const hipError_t err = device_info();
    if (err != hipSuccess) return err;
  }
  if (a.llr_type != VIT_LLR_F32 && a.sub_bits == 0) {
    const int m = resolve_metric(a.k, a.beta, a.llr_type, a.metric_bits, a.max_block_stages, why);
    if (m < 0) {
      *unsupported = 1;
      return hipSuccess;
    }
    if (m == kMetric16) return launch_blocked16(a, stream, unsupported, why);
  } else if (a.llr_type != VIT_LLR_F32) {
    // subframe traceback: the exact-in-fp32 integer kernels only
    if (a.metric_bits == kMetric16) {
      *unsupported = 1;
      *why = "subframe traceback runs with 32-bit metrics only";
      return hipSuccess;
    }
    if (!fp32_integer_exact(a.beta, a.max_block_stages)) {
      *unsupported = 1;
      *why = "int8 block too long for exact integers in fp32";
      return hipSuccess;
    }
  }
  bool stdc = true;
  for (int b = 0; b < a.beta; ++b) stdc = stdc && ((a.gen[b] >> (a.k - 1)) & 1u) && (a.gen[b] & 1u);
  KernelFn fn = pick_kernel(a.k, a.beta, stdc, a.llr_type, a.sub_bits > 0);
  if (!fn) {
    *unsupported = 1;
    *why = "no kernel instance for this (k, beta)";
    return hipSuccess;
  }
  hipError_t err;
  // the parallel traceback keeps one decoded byte per core bit after the survivors
  const int64_t lds_wave = lds_bytes_per_block(a.k, a.beta, a.max_block_stages) +
                           (a.sub_bits > 0 ? (a.L + 3) / 4 * 4 : 0);
  if (lds_wave > t_dev.max_lds) {
    *unsupported = 1;
    *why = "one block's survivor storage exceeds the per-workgroup LDS";
    return hipSuccess;
  }
  // Grid: one block per wave, the hardware dispatcher refilling a CU as soon
  // as a workgroup ends, except for long blocks or low occupancy, where
  // persistent waves that loop over blocks are faster.  Measured on 2^24-bit
  // streams: one block per wave is 5-15% faster for K=7 up to L = 896 and
  // K=9 up to L = 448; persistent waves are 5-16% faster from about 1000
  // stages per block (K=5..7, L = 1024, 2048) and at 4 or fewer two-wave
  // workgroups per CU (K=9, L = 512).  Persistent waves run two per
  // workgroup where their survivor storage fits (8-25% faster than one);
  // one block per wave runs one wave per workgroup (K=7 r1/2 at L = 512:
  // 64.0 against 62.2 Gb/s; -2% to +5% for the other codes and lengths).
  int wpb = (2 * lds_wave <= t_dev.max_lds) ? 2 : 1;
  int occ = 0;
  err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, reinterpret_cast<const void *>(fn), 64 * wpb,
                                                     (size_t)lds_wave * wpb);
  if (err != hipSuccess) return err;
  if (occ < 1) occ = 1;
  const bool persistent = a.max_block_stages >= 1000 || occ <= 4;
  if (!persistent) wpb = 1;
  const size_t lds = (size_t)lds_wave * wpb;
  const int64_t need = (a.nblocks + wpb - 1) / wpb;
  int64_t grid = need;
  if (persistent) {
    grid = (int64_t)occ * t_dev.num_cu;
    if (grid >= need) grid = need;
    else grid = grid / 8 * 8;
  }
  if (grid < 1) grid = 1;
  if (lds > 65536) {
    err = hipFuncSetAttribute(reinterpret_cast<const void *>(fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
    if (err != hipSuccess) return err;
  }
  DecodeArgs args = a;
  int words = (int)(lds_wave / 4);
  void *kargs[] = {&args, &words};
  err = hipLaunchKernel(reinterpret_cast<const void *>(fn), dim3((unsigned)grid), dim3(64 * wpb), kargs, lds,
                        stream);
  if (err != hipSuccess) return err;
  return hipGetLastError();
}

unsigned batch_launch_grid(const BatchLaunch &bl, int64_t count, int64_t max_block_stages, int num_cu) {
  const int64_t units = (count + bl.items_per_wave - 1) / bl.items_per_wave;
  return batch_grid(units, (int)(bl.block / 64), max_block_stages, bl.grid, num_cu);
}

hipError_t plan_batch_launch(int k, int beta, const uint32_t *gen, int in, int metric_bits, int64_t max_block_stages,
                             int wpb, BatchLaunch *bl, int *unsupported, const char **why) {
  *unsupported = 0;
  {
    const hipError_t err = device_info();
    if (err != hipSuccess) return err;
  }
  const int metric = resolve_metric(k, beta, in, metric_bits, max_block_stages, why);
  if (metric < 0) {
    *unsupported = 1;
    return hipSuccess;
  }
  if (metric == kMetric16) {
    void *fn16 = pick_kernel16(k, beta, in, true);
    if (!fn16) {
      *unsupported = 1;
      *why = "no 16-bit metric batch kernel instance for this (k, beta)";
      return hipSuccess;
    }
    const int64_t lds_wave = lds16_bytes_per_wave(k, beta, max_block_stages);
    const size_t lds = (size_t)lds_wave * wpb;
    if ((int64_t)lds > t_dev.max_lds) {
      *unsupported = 1;
      *why = "the workgroup's survivor storage exceeds the per-workgroup LDS";
      return hipSuccess;
    }
    hipError_t err;
    if (lds > 65536) {
      err = hipFuncSetAttribute(fn16, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (err != hipSuccess) return err;
    }
    int occ = 0;
    err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn16, 64 * wpb, lds);
    if (err != hipSuccess) return err;
    if (occ < 1) occ = 1;
    bl->fn = fn16;
    bl->grid = (unsigned)(occ * t_dev.num_cu);
    bl->block = (unsigned)(64 * wpb);
    bl->lds = lds;
    bl->lds_words_per_wave = (int)(lds_wave / 4);
    bl->items_per_wave = 2;
    bl->metric_bits = kMetric16;
    return hipSuccess;
  }
  bool stdc = true;
  for (int b = 0; b < beta; ++b) stdc = stdc && ((gen[b] >> (k - 1)) & 1u) && (gen[b] & 1u);
  BatchKernelFn fn = nullptr;
  switch (k) {
    case 3: fn = pick_batch_kernel_k3(beta, stdc, in); break;
    case 4: fn = pick_batch_kernel_k4(beta, stdc, in); break;
    case 5: fn = pick_batch_kernel_k5(beta, stdc, in); break;
    case 6: fn = pick_batch_kernel_k6(beta, stdc, in); break;
    case 7: fn = pick_batch_kernel_k7(beta, stdc, in); break;
    case 8: fn = pick_batch_kernel_k8(beta, stdc, in); break;
    case 9: fn = pick_batch_kernel_k9(beta, stdc, in); break;
  }
  if (!fn) {
    *unsupported = 1;
    *why = "no batch kernel instance for this (k, beta)";
    return hipSuccess;
  }
  hipError_t err;
  const int64_t lds_wave = lds_bytes_per_block(k, beta, max_block_stages);
  const size_t lds = (size_t)lds_wave * wpb;
  if ((int64_t)lds > t_dev.max_lds) {
    *unsupported = 1;
    *why = "a block's survivor storage exceeds the per-workgroup LDS";
    return hipSuccess;
  }
  if (lds > 65536) {
    err = hipFuncSetAttribute(reinterpret_cast<const void *>(fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
    if (err != hipSuccess) return err;
  }
  int occ = 0;
  err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, reinterpret_cast<const void *>(fn), 64 * wpb, lds);
  if (err != hipSuccess) return err;
  if (occ < 1) occ = 1;
  bl->fn = reinterpret_cast<const void *>(fn);
  bl->grid = (unsigned)(occ * t_dev.num_cu);
  bl->block = (unsigned)(64 * wpb);
  bl->lds = lds;
  bl->lds_words_per_wave = (int)(lds_wave / 4);
  bl->items_per_wave = 1;
  bl->metric_bits = metric;
  return hipSuccess;
}

}  // namespace vit
