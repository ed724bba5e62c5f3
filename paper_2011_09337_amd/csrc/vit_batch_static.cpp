// vit_batch_static.cpp -- vit_decode_batch_static: the batched decode of
// vit_batch.cpp for callers that cannot allocate.
//
// The work list (header + one item per block, Sec. III per frame) is built in
// fixed host arrays and copied into `scratch`, a fixed device array of this
// file; the batch kernels then read it exactly as they read a plan's
// workspace.  Each GPU holds its own copy of `scratch`: its address on a
// device comes from hipGetSymbolAddress, taken once per device with that
// device current, and only that address is ever handed to the HIP runtime or
// the kernels (in host code the array's name is not a device address).
#include <hip/hip_runtime.h>
#include <string.h>

#include <mutex>

#include "vit.h"
#include "vit_batch_items.h"
#include "vit_guard.h"
#include "vit_internal.h"
#include "vit_shapes.h"

namespace {

constexpr int64_t kItems = VIT_STATIC_BATCH_MAX_ITEMS;
constexpr int32_t kFrames = VIT_STATIC_BATCH_MAX_FRAMES;
constexpr int64_t kStages = VIT_STATIC_BATCH_MAX_STAGES;
constexpr size_t kBytes = vit::kHeaderBytes + (size_t)kItems * sizeof(vit::WorkItem);
constexpr int kMaxDevices = 64;

}  // namespace

// The last call's work list on each GPU.
static __device__ __align__(256) uint8_t scratch[kBytes];

namespace {

using vit::api_fail;

// Host side: one lock over the fixed host arrays and the per-device addresses.
std::mutex g_mu;
void *g_dev_scratch[kMaxDevices];  // hipGetSymbolAddress(scratch) per device, nullptr until taken
alignas(256) uint8_t g_host[kBytes];
vit::WorkItem g_sort_tmp[kItems];
int64_t g_sort_hist[kStages + 2];
std::pair<int64_t, int64_t> g_out_ranges[kFrames];

int decode_batch_static_impl(const vit_code *codes, int32_t ncodes, const vit_frame *frames, int32_t nframes,
                             const void *llr, int64_t llr_count, int32_t llr_type, uint8_t *out, int64_t out_bytes,
                             const vit_tuning *tune, void *stream) {
  vit::api_clear_error();
  int st = vit::check_batch_args(codes, ncodes, frames, nframes);
  if (st) return st;
  if (!llr || !out) return api_fail(VIT_EINVAL, "NULL buffer");
  if (llr_type != VIT_LLR_F32 && llr_type != VIT_LLR_I8 && llr_type != VIT_LLR_HARD)
    return api_fail(VIT_EINVAL, "unknown llr_type %d", llr_type);
  if (nframes > kFrames)
    return api_fail(VIT_EUNSUPPORTED, "%d frames: the static work list takes at most %d (VIT_STATIC_BATCH_MAX_FRAMES)",
                    nframes, kFrames);
  vit_tuning shape[vit::kMaxCodes];
  for (int c = 0; c < ncodes; ++c) {
    shape[c] = tune ? tune[c] : vit::default_tuning(codes[c]);
    st = vit::check_tuning(shape[c]);
    if (st) return st;
    if ((int64_t)shape[c].L + shape[c].v > kStages)
      return api_fail(VIT_EUNSUPPORTED, "code %d: L + v = %lld stages per block, at most %lld (VIT_STATIC_BATCH_MAX_STAGES)",
                      c, (long long)shape[c].L + shape[c].v, (long long)kStages);
    st = vit::integer_shape_precheck(codes[c].k, codes[c].beta, llr_type, vit::kMetricAuto,
                                     (int64_t)shape[c].L + shape[c].v, false);
    if (st) return st;
  }

  std::lock_guard<std::mutex> lock(g_mu);
  st = vit::check_frames(codes, ncodes, frames, nframes, llr_count, llr_type, out_bytes, g_out_ranges);
  if (st) return st;
  const int elem = llr_type == VIT_LLR_F32 ? 4 : 1;
  const int64_t total =
      vit::build_items(codes, ncodes, frames, nframes, shape, elem, nullptr, nullptr, nullptr, nullptr, nullptr);
  if (total > kItems)
    return api_fail(VIT_EUNSUPPORTED, "%lld blocks: the static work list holds at most %lld (VIT_STATIC_BATCH_MAX_ITEMS)",
                    (long long)total, (long long)kItems);
  int32_t *header = (int32_t *)g_host;
  memset(header, 0, vit::kHeaderBytes);
  int64_t max_stages[vit::kMaxCodes];
  vit::build_items(codes, ncodes, frames, nframes, shape, elem, (vit::WorkItem *)(g_host + vit::kHeaderBytes), header,
                   max_stages, g_sort_tmp, g_sort_hist);
  const size_t need = vit::kHeaderBytes + (size_t)total * sizeof(vit::WorkItem);

  // ---- device work: this device's copy of `scratch`
  int dev = 0;
  hipError_t he = hipGetDevice(&dev);
  if (he != hipSuccess) return vit::api_fail_hip(he, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return api_fail(VIT_EUNSUPPORTED, "device %d: at most %d devices", dev, kMaxDevices);
  if (!g_dev_scratch[dev]) {
    void *p = nullptr;
    he = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (he != hipSuccess) return vit::api_fail_hip(he, "hipGetSymbolAddress(scratch)");
    g_dev_scratch[dev] = p;
  }
  uint8_t *ws = (uint8_t *)g_dev_scratch[dev];
  int ncu = 256;
  he = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (he != hipSuccess) return vit::api_fail_hip(he, "hipDeviceGetAttribute");

  // plan every code's launch before any device work, so that an unsupported
  // shape leaves the device untouched
  vit::BatchLaunch bl[vit::kMaxCodes];
  for (int c = 0; c < ncodes; ++c) {
    int unsupported = 0;
    const char *why = "";
    he = vit::plan_batch_launch(codes[c].k, codes[c].beta, codes[c].gen, llr_type, vit::kMetricAuto,
                                (int64_t)shape[c].L + shape[c].v, shape[c].waves_per_block, &bl[c], &unsupported,
                                &why);
    if (he != hipSuccess) return vit::api_fail_hip(he, "batch launch planning");
    if (unsupported) return api_fail(VIT_EUNSUPPORTED, "code %d: %s", c, why);
  }

  // The copy is ordered after earlier work on `stream` (which may still read
  // the array); waiting for it frees the host arrays for the next call.
  he = hipMemcpyAsync(ws, g_host, need, hipMemcpyHostToDevice, (hipStream_t)stream);
  if (he != hipSuccess) return vit::api_fail_hip(he, "hipMemcpyAsync(work list)");
  he = hipStreamSynchronize((hipStream_t)stream);
  if (he != hipSuccess) return vit::api_fail_hip(he, "hipStreamSynchronize");

  int order[vit::kMaxCodes];
  vit::batch_code_order(codes, ncodes, order);
  for (int oi = 0; oi < ncodes; ++oi) {
    const int c = order[oi];
    if (header[vit::kMaxCodes + c] == 0) continue;
    vit::BatchArgs args;
    args.llr = llr;
    args.out = out;
    args.header = (int32_t *)ws;
    args.items = (const vit::WorkItem *)(ws + vit::kHeaderBytes);
    args.code_index = c;
    for (int b = 0; b < 4; ++b) args.gen[b] = b < codes[c].beta ? codes[c].gen[b] : 0u;
    int words = bl[c].lds_words_per_wave;
    void *kargs[] = {&args, &words};
    const unsigned grid =
        vit::batch_launch_grid(bl[c], header[vit::kMaxCodes + c], (int64_t)shape[c].L + shape[c].v, ncu);
    he = hipLaunchKernel(bl[c].fn, dim3(grid), dim3(bl[c].block), kargs, bl[c].lds, (hipStream_t)stream);
    if (he != hipSuccess) return vit::api_fail_hip(he, "batch kernel launch");
  }
  he = hipGetLastError();
  if (he != hipSuccess) return vit::api_fail_hip(he, "batch kernel launch");
  return VIT_OK;
}

}  // namespace

extern "C" int vit_decode_batch_static(const vit_code *codes, int32_t ncodes, const vit_frame *frames,
                                       int32_t nframes, const void *llr, int64_t llr_count, int32_t llr_type,
                                       uint8_t *out, int64_t out_bytes, const vit_tuning *tune, void *stream) {
  return vit::guard_entry("vit_decode_batch_static", [&] {
    return decode_batch_static_impl(codes, ncodes, frames, nframes, llr, llr_count, llr_type, out, out_bytes, tune,
                                    stream);
  });
}
