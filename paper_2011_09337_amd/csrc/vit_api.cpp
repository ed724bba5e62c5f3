// vit_api.cpp -- the C ABI declared in include/vit.h: argument validation,
// block geometry (Sec. III of the paper) and kernel launch.
//
// Validation happens entirely on the host before any HIP call, so argument
// errors are reported without touching a device.
#include "vit.h"

#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <atomic>

#include "vit_check.h"
#include "vit_guard.h"
#include "vit_internal.h"

namespace {
thread_local char t_err[512] = "";
}  // namespace

namespace vit {

void api_clear_error() { t_err[0] = 0; }

int api_fail(int status, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(t_err, sizeof(t_err), fmt, ap);
  va_end(ap);
  return status;
}

int api_fail_hip(hipError_t e, const char *what) {
  return api_fail(VIT_EDEVICE, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
}

// Pending allocation failures requested by vit_debug_fail_allocations.
static std::atomic<int32_t> g_fail_allocs{0};

bool alloc_checkpoint_fails() {
  int32_t n = g_fail_allocs.load(std::memory_order_relaxed);
  while (n > 0 && !g_fail_allocs.compare_exchange_weak(n, n - 1, std::memory_order_relaxed)) {
  }
  return n > 0;
}

}  // namespace vit

namespace {

using vit::api_fail;
int fail(int status, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int status, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(t_err, sizeof(t_err), fmt, ap);
  va_end(ap);
  return status;
}

int fail_hip(hipError_t e, const char *what) { return vit::api_fail_hip(e, what); }

int check_code(const vit_code *c) {
  if (!c) return fail(VIT_EINVAL, "code is NULL");
  if (c->k < 3 || c->k > 9) return fail(VIT_EINVAL, "k = %d outside [3, 9]", c->k);
  if (c->beta < 2 || c->beta > 4) return fail(VIT_EINVAL, "beta = %d outside [2, 4]", c->beta);
  for (int b = 0; b < c->beta; ++b) {
    if (c->gen[b] == 0 || c->gen[b] >= (1u << c->k))
      return fail(VIT_EINVAL, "generator %d = %u outside (0, 2^k)", b, c->gen[b]);
  }
  return VIT_OK;
}

}  // namespace

namespace vit {
int api_check_code(const vit_code *c) { return check_code(c); }

int integer_shape_precheck(int k, int beta, int llr_type, int metric_bits, int64_t max_block_stages, bool subframes) {
  if (llr_type == VIT_LLR_F32) return VIT_OK;
  // gfx950 has 160 KiB of LDS per workgroup; the launch checks the device's own figure
  const int64_t lds_cap = 160 * 1024;
  const bool fits16 = !subframes && lds16_bytes_per_wave(k, beta, max_block_stages) <= lds_cap;
  const bool fits32 = fp32_integer_exact(beta, max_block_stages);
  if (metric_bits == kMetric32 && !fits32)
    return api_fail(VIT_EUNSUPPORTED, "int8 block of %lld stages: integers exact in fp32 only below 2^24 / (128 beta)",
                    (long long)max_block_stages);
  if (metric_bits == kMetric16 && !fits16)
    return api_fail(VIT_EUNSUPPORTED, "int8 block of %lld stages: %s", (long long)max_block_stages,
                    subframes ? "subframe traceback runs with 32-bit metrics only"
                              : "two blocks' survivors exceed the LDS of a workgroup");
  if (metric_bits == kMetricAuto && !fits16 && !fits32)
    return api_fail(VIT_EUNSUPPORTED, "int8 block of %lld stages fits neither integer kernel", (long long)max_block_stages);
  return VIT_OK;
}
}  // namespace vit

namespace {

struct Geometry {
  int64_t N, L, v1, v2, nblocks, max_block_stages;
};

// Block b: core [bL, min((b+1)L, n)), stages [max(0, bL - v1), min(N, core_end + v2)).
// L = 0 is the full frame: one block over all N stages.
int resolve(const vit_code *code, int64_t n, int32_t L, int32_t v, int32_t v1_in, int32_t terminated,
            Geometry *g) {
  int st = check_code(code);
  if (st) return st;
  if (n <= 0) return fail(VIT_EINVAL, "n = %lld must be positive", (long long)n);
  if (L < 0) return fail(VIT_EINVAL, "L = %d must be >= 0", L);
  if (v < 0) return fail(VIT_EINVAL, "v = %d must be >= 0", v);
  if (v1_in > v) return fail(VIT_EINVAL, "v1 = %d exceeds v = %d", v1_in, v);
  if (terminated != 0 && terminated != 1) return fail(VIT_EINVAL, "terminated must be 0 or 1");
  g->N = n + (terminated ? code->k - 1 : 0);
  if (L == 0) {
    g->L = n;
    g->v1 = 0;
    g->v2 = g->N - n;
  } else {
    g->L = L;
    g->v1 = v1_in < 0 ? v / 2 : v1_in;
    g->v2 = v - g->v1;
  }
  g->nblocks = (n + g->L - 1) / g->L;
  // every block spans at most L + v1 + v2 stages (fewer where clipped to the stream)
  const int64_t mx = g->L + g->v1 + g->v2 < g->N ? g->L + g->v1 + g->v2 : g->N;
  g->max_block_stages = mx;
  if (mx > (int64_t)1 << 30) return fail(VIT_EUNSUPPORTED, "block of %lld stages is too long", (long long)mx);
  return VIT_OK;
}

}  // namespace

extern "C" {

const char *vit_last_error(void) { return t_err; }

int vit_abi_version(void) { return VIT_ABI_VERSION; }

int vit_debug_fail_allocations(int32_t count) {
  vit::api_clear_error();
  if (count < 0) return api_fail(VIT_EINVAL, "count = %d < 0", count);
  vit::g_fail_allocs.store(count);
  return VIT_OK;
}

vit_opts vit_opts_default(void) {
  vit_opts o;
  memset(&o, 0, sizeof(o));
  o.size = sizeof(vit_opts);
  o.llr_type = VIT_LLR_F32;
  o.terminated = 1;
  o.v1 = -1;
  o.check_finite = 0;
  o.stream = nullptr;
  o.subframe_bits = 0;
  o.subframe_overlap = 0;
  o.subframe_start = VIT_SUBFRAME_STORED;
  o.subframe_seed = 0;
  o.metric_bits = 0;
  return o;
}

int vit_query_geometry(const vit_code *code, int64_t n, int32_t L, int32_t v, int32_t v1, int32_t terminated,
                       vit_geometry *geo) {
  t_err[0] = 0;
  if (!geo) return fail(VIT_EINVAL, "geo is NULL");
  Geometry g;
  const int st = resolve(code, n, L, v, v1, terminated, &g);
  if (st) return st;
  geo->n_stages = g.N;
  geo->n_blocks = g.nblocks;
  geo->v1 = g.v1;
  geo->v2 = g.v2;
  int64_t total = 0;
  for (int64_t b = 0; b < g.nblocks; ++b) {
    const int64_t cs = b * g.L, ce = cs + g.L < n ? cs + g.L : n;
    const int64_t s = cs - g.v1 > 0 ? cs - g.v1 : 0, e = ce + g.v2 < g.N ? ce + g.v2 : g.N;
    total += e - s;
  }
  geo->stages_total = total;
  geo->max_block_stages = g.max_block_stages;
  geo->lds_bytes_per_block = vit::lds_bytes_per_block(code->k, code->beta, g.max_block_stages);
  return VIT_OK;
}

static int decode_ex_impl(const vit_code *code, const void *llr, int64_t n, int32_t L, int32_t v,
                          int32_t tie_rule, uint8_t *out_bits, const vit_opts *opts) {
  t_err[0] = 0;
  vit_opts o = vit_opts_default();
  if (opts) {
    if (opts->size != sizeof(vit_opts)) return fail(VIT_EINVAL, "opts->size = %u, expected %zu", opts->size,
                                                    sizeof(vit_opts));
    o = *opts;
  }
  if (tie_rule != VIT_TIE_LOWER_PRED) return fail(VIT_EINVAL, "unknown tie rule %d", tie_rule);
  if (!llr) return fail(VIT_EINVAL, "llr is NULL");
  if (!out_bits) return fail(VIT_EINVAL, "out_bits is NULL");
  if (o.llr_type != VIT_LLR_F32 && o.llr_type != VIT_LLR_I8 && o.llr_type != VIT_LLR_HARD)
    return fail(VIT_EINVAL, "unknown llr_type %d", o.llr_type);
  if (o.check_finite != 0 && o.check_finite != 1) return fail(VIT_EINVAL, "check_finite = %d (0 or 1)", o.check_finite);
  if (o.metric_bits != 0 && o.metric_bits != 16 && o.metric_bits != 32)
    return fail(VIT_EINVAL, "metric_bits = %d (0, 16 or 32)", o.metric_bits);
  if (o.subframe_bits < 0) return fail(VIT_EINVAL, "subframe_bits = %d must be >= 0", o.subframe_bits);
  if (o.subframe_bits > 0 && (o.subframe_overlap < 0 || o.subframe_overlap > (1 << 24)))
    return fail(VIT_EINVAL, "subframe_overlap = %d outside [0, 2^24]", o.subframe_overlap);
  if (o.subframe_bits > 0 && o.subframe_start != VIT_SUBFRAME_STORED && o.subframe_start != VIT_SUBFRAME_RANDOM)
    return fail(VIT_EINVAL, "unknown subframe_start %d", o.subframe_start);
  Geometry g;
  int st = resolve(code, n, L, v, o.v1, o.terminated, &g);
  if (st) return st;
  if (L > 0 && (L % 8) != 0) return fail(VIT_EUNSUPPORTED, "L = %d must be a multiple of 8", L);
  // the kernels address LLRs with 32-bit byte offsets inside the stream
  const int64_t llr_bytes = g.N * code->beta * (o.llr_type == VIT_LLR_F32 ? 4 : 1);
  if (llr_bytes >= ((int64_t)1 << 32) || g.N >= ((int64_t)1 << 31))
    return fail(VIT_EUNSUPPORTED, "stream of %lld LLR bytes is too long (limit 2^32)", (long long)llr_bytes);
  st = vit::integer_shape_precheck(code->k, code->beta, o.llr_type, o.metric_bits, g.max_block_stages,
                                   o.subframe_bits > 0);
  if (st) return st;
  vit::DecodeArgs a;
  a.llr = llr;
  a.out = out_bits;
  a.n = n;
  a.N = g.N;
  a.L = g.L;
  a.v1 = g.v1;
  a.v2 = g.v2;
  a.nblocks = g.nblocks;
  for (int b = 0; b < 4; ++b) a.gen[b] = b < code->beta ? code->gen[b] : 0;
  a.k = code->k;
  a.beta = code->beta;
  a.terminated = o.terminated;
  a.llr_type = o.llr_type;
  a.max_block_stages = (int32_t)g.max_block_stages;
  a.sub_bits = o.subframe_bits;
  a.sub_overlap = o.subframe_bits > 0 ? o.subframe_overlap : 0;
  a.sub_start = o.subframe_bits > 0 ? o.subframe_start : VIT_SUBFRAME_STORED;
  a.sub_seed = o.subframe_seed;
  a.metric_bits = o.metric_bits;
  // one lane per subframe chain: at most 64 subframes of the longest core
  if (o.subframe_bits > 0 && (g.L + o.subframe_bits - 1) / o.subframe_bits > 64)
    return fail(VIT_EUNSUPPORTED, "cores of %lld bits in subframes of %d: more than 64 subframes per block",
                (long long)g.L, o.subframe_bits);
  if (o.check_finite && o.llr_type == VIT_LLR_F32) {
    int nonfinite = 0;
    const hipError_t ce = vit::check_finite_f32((const float *)llr, g.N * code->beta, (hipStream_t)o.stream, &nonfinite);
    if (ce != hipSuccess) return fail_hip(ce, "finiteness pre-pass");
    if (nonfinite) return fail(VIT_EINVAL, "an LLR is NaN or infinite");
  }
  int unsupported = 0;
  const char *why = "";
  hipError_t e = vit::launch_blocked(a, (hipStream_t)o.stream, &unsupported, &why);
  if (e != hipSuccess) return fail_hip(e, "launch");
  if (unsupported) return fail(VIT_EUNSUPPORTED, "%s", why);
  return VIT_OK;
}

int vit_decode_ex(const vit_code *code, const void *llr, int64_t n, int32_t L, int32_t v, int32_t tie_rule,
                  uint8_t *out_bits, const vit_opts *opts) {
  return vit::guard_entry("vit_decode_ex", [&] { return decode_ex_impl(code, llr, n, L, v, tie_rule, out_bits, opts); });
}

int vit_depuncture(const void *received, int64_t received_count, int32_t llr_type, const uint8_t *mask,
                   int32_t period, int32_t beta, int64_t stages, void *out, void *stream) {
  t_err[0] = 0;
  if (llr_type != VIT_LLR_F32 && llr_type != VIT_LLR_I8) return fail(VIT_EINVAL, "llr_type %d (F32 or I8)", llr_type);
  if (!mask) return fail(VIT_EINVAL, "mask is NULL");
  if (beta < 2 || beta > 4) return fail(VIT_EINVAL, "beta = %d outside [2, 4]", beta);
  if (period < 1 || period * beta > 64) return fail(VIT_EINVAL, "period x beta = %d x %d outside [1, 64]", period, beta);
  if (stages < 0 || received_count < 0) return fail(VIT_EINVAL, "negative size");
  uint64_t bits = 0;
  int32_t kept = 0;
  for (int i = 0; i < period * beta; ++i)
    if (mask[i]) {
      bits |= 1ull << i;
      ++kept;
    }
  if (kept == 0) return fail(VIT_EINVAL, "the pattern keeps no output");
  // received values: whole periods, then the kept slots of the partial period
  const int64_t whole = stages / period;
  int64_t expect = whole * kept;
  for (int i = 0; i < (int)(stages - whole * period) * beta; ++i) expect += mask[i] ? 1 : 0;
  if (expect != received_count)
    return fail(VIT_EINVAL, "%lld received values, the pattern keeps %lld in %lld stages", (long long)received_count,
                (long long)expect, (long long)stages);
  if (stages > 0 && (!received || !out)) return fail(VIT_EINVAL, "NULL buffer");
  if (stages * beta >= ((int64_t)1 << 40)) return fail(VIT_EUNSUPPORTED, "stream too long");
  hipError_t e = vit::launch_depuncture(received, llr_type, bits, period, beta, kept, stages, out, (hipStream_t)stream);
  if (e != hipSuccess) return fail_hip(e, "depuncture launch");
  return VIT_OK;
}

int vit_quantize_i8(const float *llr, int64_t count, float scale, int8_t *q, void *stream) {
  t_err[0] = 0;
  if (count < 0) return fail(VIT_EINVAL, "count = %lld must be >= 0", (long long)count);
  if (count > 0 && (!llr || !q)) return fail(VIT_EINVAL, "NULL buffer");
  if (!(scale > 0.0f) || scale > 3.0e38f) return fail(VIT_EINVAL, "scale must be positive and finite");
  const hipError_t e = vit::launch_quantize(llr, count, scale, q, (hipStream_t)stream);
  if (e != hipSuccess) return fail_hip(e, "quantize launch");
  return VIT_OK;
}

int vit_decode(const vit_code *code, const float *llr, int64_t n, int32_t L, int32_t v, int32_t tie_rule,
               uint8_t *out_bits) {
  vit_opts o = vit_opts_default();
  const int st = vit_decode_ex(code, llr, n, L, v, tie_rule, out_bits, &o);
  if (st) return st;
  const hipError_t e = hipStreamSynchronize(nullptr);
  if (e != hipSuccess) return fail_hip(e, "hipStreamSynchronize");
  return VIT_OK;
}

}  // extern "C"
