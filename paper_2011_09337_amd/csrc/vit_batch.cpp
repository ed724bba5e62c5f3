// vit_batch.cpp -- batched decoding of many frames (mixed codes and lengths):
// work lists, one reusable hipGraph per plan, and the autotuner.
//
// A batch is cut into blocks exactly as each frame would be on its own
// (Sec. III of the paper, per frame).  Each block is one work item; items of
// one code are sorted by cost (stages) so that the kernel's waves take the
// longest first.  Per call the host writes the header (item
// counts and run offsets per code) and the items into pinned staging memory;
// the graph copies them into the caller's device workspace and runs one kernel
// node per code, in sequence.  While the buffers, codes and shapes stay the
// same the graph is reused; only its copy node and the kernel grids (sized to
// each code's item count) are updated.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <string>
#include <vector>

#include "vit.h"
#include "vit_batch_items.h"
#include "vit_guard.h"
#include "vit_internal.h"
#include "vit_shapes.h"

struct vit_plan {
  void *staging[2] = {nullptr, nullptr};
  size_t staging_cap[2] = {0, 0};
  hipEvent_t done[2] = {nullptr, nullptr};
  bool pending[2] = {false, false};
  int slot = 0;

  // graph cache
  bool have_graph = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraphNode_t copy_node = nullptr;                   // the header
  hipGraphNode_t code_copy[vit::kMaxCodes] = {};         // each code's run of work items
  // per code: its kernel node, launch shape, arguments and current grid
  hipGraphNode_t knode[vit::kMaxCodes] = {};
  vit::BatchLaunch bl[vit::kMaxCodes] = {};
  vit::BatchArgs kargs[vit::kMaxCodes] = {};
  int kwords[vit::kMaxCodes] = {};
  unsigned kgrid[vit::kMaxCodes] = {};
  struct Key {
    const void *llr = nullptr;
    void *out = nullptr;
    void *ws = nullptr;
    int llr_type = -1;
    int metric_bits = -1;
    int ncodes = 0;
    int dev = -1;
    vit_code codes[vit::kMaxCodes];
    vit_tuning tune[vit::kMaxCodes];
  } key;

  int metric_bits = 0;  // integer inputs: 0 (32-bit where it fits, else 16-bit), 16 or 32
  // autotuner: the largest fraction of a code's bits in which an accepted
  // shape's decode may differ from the long-overlap reference decode.  On
  // the batched configuration's Eb/N0 mix (1-5 dB) shapes that sit 0.04-0.08
  // dB from maximum likelihood at BER 1e-4 differ in about 5e-4 of the bits,
  // K=9 at v = 45 (0.15 dB) in 9.2e-4: the default admits the former only.
  double tune_tolerance = 8e-4;

  // autotuned shapes by (code, LLR type, frame-length bucket)
  std::map<std::string, vit_tuning_entry> tuned;

  // host scratch reused across calls (large per-call vectors would be mmap'd
  // and page-faulted afresh every call)
  std::vector<vit::WorkItem> sort_tmp;
  std::vector<int64_t> sort_hist;
  std::vector<std::pair<int64_t, int64_t>> out_ranges;
};

namespace vit {

static bool same_code(const vit_code &a, const vit_code &b) {
  if (a.k != b.k || a.beta != b.beta) return false;
  for (int i = 0; i < a.beta; ++i)
    if (a.gen[i] != b.gen[i]) return false;
  return true;
}

static bool same_tuning(const vit_tuning &a, const vit_tuning &b) {
  return a.L == b.L && a.v == b.v && a.v1 == b.v1 && a.waves_per_block == b.waves_per_block;
}

vit_tuning default_tuning(const vit_code &c) {
  vit_tuning t;
  t.L = 256;
  t.v = vit::default_overlap(c.k);
  t.v1 = -1;
  t.waves_per_block = 1;
  return t;
}

int check_tuning(const vit_tuning &t) {
  if (t.L <= 0 || t.L % 8 != 0) return api_fail(VIT_EINVAL, "tuning L = %d must be a positive multiple of 8", t.L);
  if (t.v < 0) return api_fail(VIT_EINVAL, "tuning v = %d must be >= 0", t.v);
  if (t.v1 < -1 || t.v1 > t.v) return api_fail(VIT_EINVAL, "tuning v1 = %d outside [-1, v]", t.v1);
  if (t.waves_per_block < 1 || t.waves_per_block > 4)
    return api_fail(VIT_EINVAL, "waves_per_block = %d outside [1, 4]", t.waves_per_block);
  return VIT_OK;
}

static int frame_bucket(int64_t mean_n) {
  int b = 0;
  while (b < 40 && ((int64_t)1 << (b + 1)) <= mean_n) ++b;
  return b;
}

static std::string tune_key(const vit_code &c, int llr_type, int bucket) {
  char buf[128];
  snprintf(buf, sizeof(buf), "k%d b%d g%u,%u,%u,%u t%d n%d", c.k, c.beta, c.gen[0], c.gen[1],
           c.beta > 2 ? c.gen[2] : 0u, c.beta > 3 ? c.gen[3] : 0u, llr_type, bucket);
  return buf;
}

int check_batch_args(const vit_code *codes, int32_t ncodes, const vit_frame *frames, int32_t nframes) {
  if (!codes || ncodes < 1 || ncodes > kMaxCodes) return api_fail(VIT_EINVAL, "ncodes = %d outside [1, 8]", ncodes);
  for (int c = 0; c < ncodes; ++c) {
    const int st = vit::api_check_code(&codes[c]);
    if (st) return st;
  }
  if (!frames || nframes < 1) return api_fail(VIT_EINVAL, "no frames");
  return VIT_OK;
}

// Work items of every frame under the given shapes.  Returns the number of
// items per code in counts[], fills header offsets, and (if items != NULL)
// the items themselves, each code's run sorted by cost, longest first.
int64_t build_items(const vit_code *codes, int32_t ncodes, const vit_frame *frames, int32_t nframes,
                    const vit_tuning *shape, int elem_bytes, WorkItem *items, int32_t *header,
                    int64_t *max_stages, WorkItem *tmp, int64_t *hist) {
  int64_t counts[kMaxCodes] = {0};
  for (int32_t f = 0; f < nframes; ++f) {
    const int c = frames[f].code_id;
    counts[c] += (frames[f].n + shape[c].L - 1) / shape[c].L;
  }
  int64_t offs[kMaxCodes] = {0};
  int64_t total = 0;
  for (int c = 0; c < ncodes; ++c) {
    offs[c] = total;
    total += counts[c];
    if (max_stages) max_stages[c] = 0;
  }
  if (!items) return total;
  int64_t fill[kMaxCodes];
  for (int c = 0; c < ncodes; ++c) fill[c] = offs[c];
  for (int32_t f = 0; f < nframes; ++f) {
    const vit_frame &fr = frames[f];
    const int c = fr.code_id;
    const vit_code &code = codes[c];
    const int64_t N = fr.n + (fr.terminated ? code.k - 1 : 0);
    const int64_t L = shape[c].L;
    const int64_t v1 = shape[c].v1 < 0 ? shape[c].v / 2 : shape[c].v1;
    const int64_t v2 = shape[c].v - v1;
    for (int64_t cs = 0; cs < fr.n; cs += L) {
      const int64_t ce = cs + L < fr.n ? cs + L : fr.n;
      const int64_t s = cs - v1 > 0 ? cs - v1 : 0;
      const int64_t e = ce + v2 < N ? ce + v2 : N;
      WorkItem &it = items[fill[c]++];
      it.llr_off = fr.llr_off * elem_bytes;
      it.out_off = fr.out_off;
      it.s = (int32_t)s;
      it.e = (int32_t)e;
      it.cs = (int32_t)cs;
      it.ce = (int32_t)ce;
      it.flags = (s == 0 ? 1 : 0) | ((fr.terminated && e == N) ? 2 : 0);
      it.cost = (int32_t)(e - s);
      if (max_stages && e - s > max_stages[c]) max_stages[c] = e - s;
    }
  }
  // each code's run longest first: a stable counting sort on the cost
  // (at most L + v stages), linear in the item count; tmp holds the longest
  // run, hist max_stages + 2 counters
  for (int c = 0; c < ncodes; ++c) {
    WorkItem *run = items + offs[c];
    const int64_t cnt = counts[c];
    if (cnt > 1) {
      int32_t maxc = 0;
      for (int64_t i = 0; i < cnt; ++i) maxc = std::max(maxc, run[i].cost);
      std::fill(hist, hist + maxc + 2, (int64_t)0);
      for (int64_t i = 0; i < cnt; ++i) ++hist[maxc - run[i].cost + 1];
      for (int32_t i = 1; i < maxc + 2; ++i) hist[i] += hist[i - 1];
      for (int64_t i = 0; i < cnt; ++i) tmp[hist[maxc - run[i].cost]++] = run[i];
      std::copy(tmp, tmp + cnt, run);
    }
    header[kMaxCodes + c] = (int32_t)counts[c];
    header[2 * kMaxCodes + c] = (int32_t)offs[c];
  }
  return total;
}

int check_frames(const vit_code *codes, int32_t ncodes, const vit_frame *frames, int32_t nframes, int64_t llr_count,
                 int llr_type, int64_t out_bytes, std::pair<int64_t, int64_t> *outs) {
  const int elem = llr_type == VIT_LLR_F32 ? 4 : 1;
  for (int32_t f = 0; f < nframes; ++f) {
    const vit_frame &fr = frames[f];
    if (fr.code_id < 0 || fr.code_id >= ncodes) return api_fail(VIT_EINVAL, "frame %d: code_id %d", f, fr.code_id);
    if (fr.n <= 0) return api_fail(VIT_EINVAL, "frame %d: n = %lld", f, (long long)fr.n);
    if (fr.terminated != 0 && fr.terminated != 1) return api_fail(VIT_EINVAL, "frame %d: terminated", f);
    if (fr.llr_off < 0 || fr.out_off < 0) return api_fail(VIT_EINVAL, "frame %d: negative offset", f);
    const vit_code &c = codes[fr.code_id];
    const int64_t N = fr.n + (fr.terminated ? c.k - 1 : 0);
    if (fr.llr_off + N * c.beta > llr_count)
      return api_fail(VIT_EINVAL, "frame %d: LLRs [%lld, %lld) beyond the buffer (%lld)", f, (long long)fr.llr_off,
                      (long long)(fr.llr_off + N * c.beta), (long long)llr_count);
    if (N * c.beta * elem >= ((int64_t)1 << 31) || fr.llr_off * elem >= ((int64_t)1 << 62))
      return api_fail(VIT_EUNSUPPORTED, "frame %d is too long", f);
    const int64_t nb = (fr.n + 7) / 8;
    if (fr.out_off + nb > out_bytes) return api_fail(VIT_EINVAL, "frame %d: output beyond the buffer", f);
    outs[f] = std::make_pair(fr.out_off, fr.out_off + nb);
  }
  // frames usually come with increasing outputs: sort only when they do not
  // (std::sort works in place)
  if (!std::is_sorted(outs, outs + nframes)) std::sort(outs, outs + nframes);
  for (int32_t i = 1; i < nframes; ++i)
    if (outs[i].first < outs[i - 1].second) return api_fail(VIT_EINVAL, "frames' output ranges overlap");
  return VIT_OK;
}

// Kernel order of a batch: the code with the most work per bit (states x rate)
// first; measured faster than running the codes' kernels side by side.
void batch_code_order(const vit_code *codes, int32_t ncodes, int *order) {
  for (int c = 0; c < ncodes; ++c) order[c] = c;
  std::stable_sort(order, order + ncodes, [&](int x, int y) {
    return ((int64_t)codes[x].beta << (codes[x].k - 1)) > ((int64_t)codes[y].beta << (codes[y].k - 1));
  });
}

}  // namespace vit

namespace {

using vit::api_fail;
using vit::kHeaderBytes;
using vit::kMaxCodes;
using vit::WorkItem;
using vit::build_items;
using vit::check_frames;
using vit::check_tuning;
using vit::default_tuning;
using vit::same_code;
using vit::same_tuning;
using vit::frame_bucket;
using vit::tune_key;

int check_args(const vit_code *codes, int32_t ncodes, const vit_frame *frames, int32_t nframes) {
  return vit::check_batch_args(codes, ncodes, frames, nframes);
}

// check_frames with the plan's range list as storage
int check_frames_plan(vit_plan *plan, const vit_code *codes, int32_t ncodes, const vit_frame *frames,
                      int32_t nframes, int64_t llr_count, int llr_type, int64_t out_bytes) {
  vit::alloc_checkpoint();
  plan->out_ranges.resize((size_t)nframes);
  return check_frames(codes, ncodes, frames, nframes, llr_count, llr_type, out_bytes, plan->out_ranges.data());
}

// build_items with the plan's sort buffers, sized for the largest run and cost
int64_t build_items_plan(vit_plan *plan, const vit_code *codes, int32_t ncodes, const vit_frame *frames,
                         int32_t nframes, const vit_tuning *shape, int elem_bytes, WorkItem *items, int32_t *header,
                         int64_t *max_stages) {
  int64_t counts[kMaxCodes] = {0};
  for (int32_t f = 0; f < nframes; ++f) counts[frames[f].code_id] += (frames[f].n + shape[frames[f].code_id].L - 1) / shape[frames[f].code_id].L;
  int64_t run = 0, cost = 0;
  for (int c = 0; c < ncodes; ++c) {
    run = std::max(run, counts[c]);
    cost = std::max(cost, (int64_t)shape[c].L + shape[c].v);
  }
  plan->sort_tmp.resize((size_t)run);
  plan->sort_hist.resize((size_t)cost + 2);
  return build_items(codes, ncodes, frames, nframes, shape, elem_bytes, items, header, max_stages,
                     plan->sort_tmp.data(), plan->sort_hist.data());
}

int resolve_shapes(vit_plan *plan, const vit_code *codes, int32_t ncodes, const vit_frame *frames, int32_t nframes,
                   int llr_type, const vit_tuning *tune, vit_tuning *shape) {
  for (int c = 0; c < ncodes; ++c) {
    if (tune) {
      shape[c] = tune[c];
    } else {
      int64_t sum = 0, cnt = 0;
      for (int32_t f = 0; f < nframes; ++f)
        if (frames[f].code_id == c) {
          sum += frames[f].n;
          ++cnt;
        }
      const int bucket = frame_bucket(cnt ? sum / cnt : 0);
      auto it = plan->tuned.find(tune_key(codes[c], llr_type, bucket));
      shape[c] = it != plan->tuned.end() ? it->second.tuning : default_tuning(codes[c]);
    }
    const int st = check_tuning(shape[c]);
    if (st) return st;
  }
  return VIT_OK;
}

int ensure_staging(vit_plan *p, int slot, size_t bytes) {
  if (p->staging_cap[slot] >= bytes) return VIT_OK;
  if (p->staging[slot]) {
    hipError_t e = hipHostFree(p->staging[slot]);
    p->staging[slot] = nullptr;
    p->staging_cap[slot] = 0;
    if (e != hipSuccess) return vit::api_fail_hip(e, "hipHostFree");
  }
  size_t cap = 1 << 16;
  while (cap < bytes) cap *= 2;
  hipError_t e = hipHostMalloc(&p->staging[slot], cap, hipHostMallocDefault);
  if (e != hipSuccess) return vit::api_fail_hip(e, "hipHostMalloc");
  p->staging_cap[slot] = cap;
  return VIT_OK;
}

// The bytes of code c's work items in the staging area and the workspace (a
// code without items copies the header again, a copy of no bytes being no
// graph node).
struct CodeCopy {
  void *dst;
  const void *src;
  size_t bytes;
};
CodeCopy code_copy_range(const int32_t *header, int c, void *workspace, const void *stg) {
  const int64_t count = header[kMaxCodes + c];
  if (count == 0) return {workspace, stg, kHeaderBytes};
  const size_t off = kHeaderBytes + (size_t)header[2 * kMaxCodes + c] * sizeof(WorkItem);
  return {(char *)workspace + off, (const char *)stg + off, (size_t)count * sizeof(WorkItem)};
}

void drop_graph(vit_plan *p) {
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  p->exec = nullptr;
  p->graph = nullptr;
  p->copy_node = nullptr;
  for (auto &n : p->code_copy) n = nullptr;
  p->have_graph = false;
}

}  // namespace

extern "C" {

int vit_plan_create(vit_plan **plan) {
  vit::api_clear_error();
  if (!plan) return api_fail(VIT_EINVAL, "plan is NULL");
  *plan = vit::alloc_checkpoint_fails() ? nullptr : new (std::nothrow) vit_plan();
  if (!*plan) return api_fail(VIT_ENOMEM, "plan allocation failed");
  return VIT_OK;
}

void vit_plan_destroy(vit_plan *plan) {
  if (!plan) return;
  for (int i = 0; i < 2; ++i) {
    if (plan->done[i]) {
      (void)hipEventSynchronize(plan->done[i]);
      (void)hipEventDestroy(plan->done[i]);
    }
    if (plan->staging[i]) (void)hipHostFree(plan->staging[i]);
  }
  drop_graph(plan);
  delete plan;
}

static int batch_workspace_size_impl(const vit_code *codes, int32_t ncodes, const vit_frame *frames,
                                     int32_t nframes, const vit_tuning *tune, size_t *bytes) {
  vit::api_clear_error();
  int st = check_args(codes, ncodes, frames, nframes);
  if (st) return st;
  if (!bytes) return api_fail(VIT_EINVAL, "bytes is NULL");
  vit_tuning shape[kMaxCodes];
  for (int c = 0; c < ncodes; ++c) {
    if (tune) {
      shape[c] = tune[c];
      st = check_tuning(shape[c]);
      if (st) return st;
    } else {
      shape[c] = default_tuning(codes[c]);
      shape[c].L = 64;  // the smallest block the autotuner tries: the most items
    }
  }
  for (int32_t f = 0; f < nframes; ++f)
    if (frames[f].code_id < 0 || frames[f].code_id >= ncodes || frames[f].n <= 0)
      return api_fail(VIT_EINVAL, "frame %d: bad code_id or n", f);
  const int64_t total = build_items(codes, ncodes, frames, nframes, shape, 4, nullptr, nullptr, nullptr, nullptr, nullptr);
  *bytes = kHeaderBytes + (size_t)total * sizeof(WorkItem);
  return VIT_OK;
}

static int decode_batch_impl(vit_plan *plan, const vit_code *codes, int32_t ncodes, const vit_frame *frames,
                             int32_t nframes, const void *llr, int64_t llr_count, int32_t llr_type, uint8_t *out,
                             int64_t out_bytes, const vit_tuning *tune, void *workspace, size_t workspace_bytes,
                             void *stream) {
  vit::api_clear_error();
  if (!plan) return api_fail(VIT_EINVAL, "plan is NULL");
  int st = check_args(codes, ncodes, frames, nframes);
  if (st) return st;
  if (!llr || !out || !workspace) return api_fail(VIT_EINVAL, "NULL buffer");
  if (((uintptr_t)workspace & 255u) != 0) return api_fail(VIT_EINVAL, "workspace must be 256-byte aligned");
  if (llr_type != VIT_LLR_F32 && llr_type != VIT_LLR_I8 && llr_type != VIT_LLR_HARD)
    return api_fail(VIT_EINVAL, "unknown llr_type %d", llr_type);
  st = check_frames_plan(plan, codes, ncodes, frames, nframes, llr_count, llr_type, out_bytes);
  if (st) return st;
  vit_tuning shape[kMaxCodes];
  st = resolve_shapes(plan, codes, ncodes, frames, nframes, llr_type, tune, shape);
  if (st) return st;
  for (int c = 0; c < ncodes; ++c) {
    st = vit::integer_shape_precheck(codes[c].k, codes[c].beta, llr_type, plan->metric_bits,
                                     (int64_t)shape[c].L + shape[c].v, false);
    if (st) return st;
  }

  const int elem = llr_type == VIT_LLR_F32 ? 4 : 1;
  const int64_t total = build_items(codes, ncodes, frames, nframes, shape, elem, nullptr, nullptr, nullptr, nullptr, nullptr);
  const size_t need = kHeaderBytes + (size_t)total * sizeof(WorkItem);
  if (workspace_bytes < need)
    return api_fail(VIT_EINVAL, "workspace of %zu bytes, %zu needed", workspace_bytes, need);
  if (total >= ((int64_t)1 << 31)) return api_fail(VIT_EUNSUPPORTED, "too many blocks");

  // the staging slot's previous copy must have run before it is rewritten
  const int slot = plan->slot;
  hipError_t he;
  if (plan->pending[slot]) {
    he = hipEventSynchronize(plan->done[slot]);
    if (he != hipSuccess) return vit::api_fail_hip(he, "hipEventSynchronize");
    plan->pending[slot] = false;
  }
  st = ensure_staging(plan, slot, need);
  if (st) return st;
  char *stg = (char *)plan->staging[slot];
  int32_t *header = (int32_t *)stg;
  memset(header, 0, kHeaderBytes);
  int64_t max_stages[kMaxCodes];
  build_items_plan(plan, codes, ncodes, frames, nframes, shape, elem, (WorkItem *)(stg + kHeaderBytes), header,
                   max_stages);

  int dev = 0;
  he = hipGetDevice(&dev);
  if (he != hipSuccess) return vit::api_fail_hip(he, "hipGetDevice");

  int ncu = 256;
  he = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (he != hipSuccess) return vit::api_fail_hip(he, "hipDeviceGetAttribute");

  // graph: reuse while buffers, codes and shapes are unchanged
  vit_plan::Key key;
  key.llr = llr;
  key.out = out;
  key.ws = workspace;
  key.llr_type = llr_type;
  key.metric_bits = plan->metric_bits;
  key.ncodes = ncodes;
  key.dev = dev;
  bool same = plan->have_graph && plan->key.llr == llr && plan->key.out == out && plan->key.ws == workspace &&
              plan->key.llr_type == llr_type && plan->key.metric_bits == plan->metric_bits &&
              plan->key.ncodes == ncodes && plan->key.dev == dev;
  for (int c = 0; c < ncodes; ++c) {
    key.codes[c] = codes[c];
    key.tune[c] = shape[c];
    if (same) same = same_code(plan->key.codes[c], codes[c]) && same_tuning(plan->key.tune[c], shape[c]);
  }
  auto grid_for = [&](int c) -> unsigned {
    return vit::batch_launch_grid(plan->bl[c], header[kMaxCodes + c], (int64_t)shape[c].L + shape[c].v, ncu);
  };
  if (!same) {
    // The old graph goes first: if planning or building fails below, no
    // later call may take the reuse branch with a half-updated plan.  The
    // launch shapes are planned aside and kept only with a complete graph.
    drop_graph(plan);
    // launch shapes (LDS sized for the longest block a shape can produce)
    vit::BatchLaunch bl[kMaxCodes];
    for (int c = 0; c < ncodes; ++c) {
      int unsupported = 0;
      const char *why = "";
      he = vit::plan_batch_launch(codes[c].k, codes[c].beta, codes[c].gen, llr_type, plan->metric_bits,
                                  (int64_t)shape[c].L + shape[c].v, shape[c].waves_per_block, &bl[c], &unsupported,
                                  &why);
      if (he != hipSuccess) return vit::api_fail_hip(he, "batch launch planning");
      if (unsupported) return api_fail(VIT_EUNSUPPORTED, "code %d: %s", c, why);
    }
    he = hipGraphCreate(&plan->graph, 0);
    if (he != hipSuccess) return vit::api_fail_hip(he, "hipGraphCreate");
    he = hipGraphAddMemcpyNode1D(&plan->copy_node, plan->graph, nullptr, 0, workspace, stg, kHeaderBytes,
                                 hipMemcpyHostToDevice);
    if (he != hipSuccess) return vit::api_fail_hip(he, "hipGraphAddMemcpyNode1D");
    // one kernel node per code, run one after another, the code with the
    // most work per bit (states x rate) first: measured faster than running
    // them side by side.  Each code's work items are copied by a node of
    // their own, the copies chained in launch order, so that a kernel waits
    // only for its own items and the later codes' copies run during the
    // earlier kernels.
    int order[kMaxCodes];
    vit::batch_code_order(codes, ncodes, order);
    hipGraphNode_t prev = nullptr, prev_copy = plan->copy_node;
    for (int oi = 0; oi < ncodes; ++oi) {
      const int c = order[oi];
      {
        const CodeCopy cc = code_copy_range(header, c, workspace, stg);
        he = hipGraphAddMemcpyNode1D(&plan->code_copy[c], plan->graph, &prev_copy, 1, cc.dst, cc.src, cc.bytes,
                                     hipMemcpyHostToDevice);
        if (he != hipSuccess) return vit::api_fail_hip(he, "hipGraphAddMemcpyNode1D");
        prev_copy = plan->code_copy[c];
      }
      vit::BatchArgs &args = plan->kargs[c];
      args.llr = llr;
      args.out = out;
      args.header = (int32_t *)workspace;
      args.items = (const WorkItem *)((char *)workspace + kHeaderBytes);
      args.code_index = c;
      for (int b = 0; b < 4; ++b) args.gen[b] = b < codes[c].beta ? codes[c].gen[b] : 0u;
      plan->kwords[c] = bl[c].lds_words_per_wave;
      void *kargs[] = {&args, &plan->kwords[c]};
      plan->kgrid[c] = vit::batch_launch_grid(bl[c], header[kMaxCodes + c], (int64_t)shape[c].L + shape[c].v, ncu);
      hipKernelNodeParams kp;
      memset(&kp, 0, sizeof(kp));
      kp.func = const_cast<void *>(bl[c].fn);
      kp.gridDim = dim3(plan->kgrid[c]);
      kp.blockDim = dim3(bl[c].block);
      kp.sharedMemBytes = (unsigned)bl[c].lds;
      kp.kernelParams = kargs;
      kp.extra = nullptr;
      hipGraphNode_t kn;
      hipGraphNode_t deps[2] = {plan->code_copy[c], prev};
      he = hipGraphAddKernelNode(&kn, plan->graph, deps, prev ? 2 : 1, &kp);
      if (he != hipSuccess) return vit::api_fail_hip(he, "hipGraphAddKernelNode");
      plan->knode[c] = kn;
      prev = kn;
    }
    he = hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0);
    if (he != hipSuccess) {
      drop_graph(plan);
      return vit::api_fail_hip(he, "hipGraphInstantiate");
    }
    for (int c = 0; c < ncodes; ++c) plan->bl[c] = bl[c];
    plan->key = key;
    plan->have_graph = true;
  } else {
    he = hipGraphExecMemcpyNodeSetParams1D(plan->exec, plan->copy_node, workspace, stg, kHeaderBytes,
                                           hipMemcpyHostToDevice);
    if (he != hipSuccess) return vit::api_fail_hip(he, "hipGraphExecMemcpyNodeSetParams1D");
    for (int c = 0; c < ncodes; ++c) {
      const CodeCopy cc = code_copy_range(header, c, workspace, stg);
      he = hipGraphExecMemcpyNodeSetParams1D(plan->exec, plan->code_copy[c], cc.dst, cc.src, cc.bytes,
                                             hipMemcpyHostToDevice);
      if (he != hipSuccess) return vit::api_fail_hip(he, "hipGraphExecMemcpyNodeSetParams1D");
    }
    // the item counts change from call to call: resize the dispatcher-refilled grids
    for (int c = 0; c < ncodes; ++c) {
      const unsigned g = grid_for(c);
      if (g == plan->kgrid[c]) continue;
      void *kargs[] = {&plan->kargs[c], &plan->kwords[c]};
      hipKernelNodeParams kp;
      memset(&kp, 0, sizeof(kp));
      kp.func = const_cast<void *>(plan->bl[c].fn);
      kp.gridDim = dim3(g);
      kp.blockDim = dim3(plan->bl[c].block);
      kp.sharedMemBytes = (unsigned)plan->bl[c].lds;
      kp.kernelParams = kargs;
      kp.extra = nullptr;
      he = hipGraphExecKernelNodeSetParams(plan->exec, plan->knode[c], &kp);
      if (he != hipSuccess) return vit::api_fail_hip(he, "hipGraphExecKernelNodeSetParams");
      plan->kgrid[c] = g;
    }
  }
  he = hipGraphLaunch(plan->exec, (hipStream_t)stream);
  if (he != hipSuccess) return vit::api_fail_hip(he, "hipGraphLaunch");
  if (!plan->done[slot]) {
    // a timing event: on this runtime recording one costs about a quarter
    // of recording an event with timing disabled
    he = hipEventCreate(&plan->done[slot]);
    if (he != hipSuccess) return vit::api_fail_hip(he, "hipEventCreate");
  }
  he = hipEventRecord(plan->done[slot], (hipStream_t)stream);
  if (he != hipSuccess) return vit::api_fail_hip(he, "hipEventRecord");
  plan->pending[slot] = true;
  plan->slot = slot ^ 1;
  return VIT_OK;
}

// Autotune (see vit.h).  Per code: decode the code's frames once with the
// reference shape (L = 512, v1 = v2 = 128, far beyond the trellis's
// convergence depth), then each candidate (L, v, waves) once; a candidate
// whose decode differs from the reference in more than tune_tolerance of the
// code's bits is rejected, the others are timed (3 runs) and the fastest is
// kept.  The outputs are compared on the host.
static int plan_autotune_impl(vit_plan *plan, const vit_code *codes, int32_t ncodes, const vit_frame *frames,
                              int32_t nframes, const void *llr, int64_t llr_count, int32_t llr_type, uint8_t *out,
                              int64_t out_bytes, void *workspace, size_t workspace_bytes, void *stream,
                              vit_tuning *chosen) {
  vit::api_clear_error();
  if (!plan) return api_fail(VIT_EINVAL, "plan is NULL");
  int st = check_args(codes, ncodes, frames, nframes);
  if (st) return st;
  st = check_frames_plan(plan, codes, ncodes, frames, nframes, llr_count, llr_type, out_bytes);
  if (st) return st;
  hipEvent_t e0, e1;
  hipError_t he = hipEventCreate(&e0);
  if (he != hipSuccess) return vit::api_fail_hip(he, "hipEventCreate");
  he = hipEventCreate(&e1);
  if (he != hipSuccess) {
    (void)hipEventDestroy(e0);
    return vit::api_fail_hip(he, "hipEventCreate");
  }
  std::vector<uint8_t> ref((size_t)out_bytes), cand((size_t)out_bytes);
  // decode the code's frames with shape t and copy the output to `host`
  auto decode_to = [&](const vit_code &code, const std::vector<vit_frame> &sub, const vit_tuning &t,
                       std::vector<uint8_t> &host) -> int {
    int r = vit_decode_batch(plan, &code, 1, sub.data(), (int32_t)sub.size(), llr, llr_count, llr_type, out,
                             out_bytes, &t, workspace, workspace_bytes, stream);
    if (r) return r;
    hipError_t e = hipMemcpyAsync(host.data(), out, (size_t)out_bytes, hipMemcpyDeviceToHost, (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    return e == hipSuccess ? VIT_OK : vit::api_fail_hip(e, "copy of a candidate's output");
  };
  static const int kL[] = {64, 128, 256, 512, 1024};
  int result = VIT_OK;
  for (int c = 0; c < ncodes && result == VIT_OK; ++c) {
    std::vector<vit_frame> sub;
    int64_t sum = 0;
    for (int32_t f = 0; f < nframes; ++f)
      if (frames[f].code_id == c) {
        sub.push_back(frames[f]);
        sub.back().code_id = 0;
        sum += frames[f].n;
      }
    vit_tuning best = default_tuning(codes[c]);
    if (sub.empty()) {
      if (chosen) chosen[c] = best;
      continue;
    }
    const int k = codes[c].k;
    vit_tuning reft;
    reft.L = 512;
    reft.v = 256;
    reft.v1 = 128;
    reft.waves_per_block = 1;
    result = decode_to(codes[c], sub, reft, ref);
    if (result) break;
    const int64_t max_diff = (int64_t)(plan->tune_tolerance * (double)sum);
    // candidate overlaps: 5k, 6k, 7k, 8(k-1), 10(k-1)
    std::vector<int> vs = {5 * k, 6 * k, 7 * k, 8 * (k - 1), 10 * (k - 1)};
    std::sort(vs.begin(), vs.end());
    vs.erase(std::unique(vs.begin(), vs.end()), vs.end());
    best = reft;  // the reference itself when no candidate meets the bound
    float best_ms = 1e30f;
    for (int li = 0; li < 5 && result == VIT_OK; ++li) {
      for (size_t vi = 0; vi < vs.size() && result == VIT_OK; ++vi) {
        for (int w = 1; w <= 2 && result == VIT_OK; ++w) {
          vit_tuning t;
          t.L = kL[li];
          t.v = vs[vi];
          t.v1 = -1;
          t.waves_per_block = w;
          st = decode_to(codes[c], sub, t, cand);
          if (st == VIT_EUNSUPPORTED) continue;  // shape does not fit: not a candidate
          if (st) {
            result = st;
            break;
          }
          int64_t diff = 0;
          for (int64_t i = 0; i < out_bytes; ++i) diff += __builtin_popcount((unsigned)(ref[i] ^ cand[i]));
          if (diff > max_diff) continue;  // too far from the reference
          (void)hipEventRecord(e0, (hipStream_t)stream);
          for (int rep = 0; rep < 3 && result == VIT_OK; ++rep)
            result = vit_decode_batch(plan, &codes[c], 1, sub.data(), (int32_t)sub.size(), llr, llr_count,
                                      llr_type, out, out_bytes, &t, workspace, workspace_bytes, stream);
          (void)hipEventRecord(e1, (hipStream_t)stream);
          he = hipEventSynchronize(e1);
          if (he != hipSuccess) {
            result = vit::api_fail_hip(he, "hipEventSynchronize");
            break;
          }
          float ms = 0;
          (void)hipEventElapsedTime(&ms, e0, e1);
          if (ms < best_ms) {
            best_ms = ms;
            best = t;
          }
        }
      }
    }
    if (result == VIT_OK) {
      const int bucket = frame_bucket(sum / (int64_t)sub.size());
      vit_tuning_entry &ent = plan->tuned[tune_key(codes[c], llr_type, bucket)];
      ent.code = codes[c];
      ent.llr_type = llr_type;
      ent.length_bucket = bucket;
      ent.tuning = best;
      if (chosen) chosen[c] = best;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return result;
}

// The entry points: no exception leaves the C ABI (vit_guard.h).
int vit_batch_workspace_size(const vit_code *codes, int32_t ncodes, const vit_frame *frames, int32_t nframes,
                             const vit_tuning *tune, size_t *bytes) {
  return vit::guard_entry("vit_batch_workspace_size",
                          [&] { return batch_workspace_size_impl(codes, ncodes, frames, nframes, tune, bytes); });
}

int vit_decode_batch(vit_plan *plan, const vit_code *codes, int32_t ncodes, const vit_frame *frames,
                     int32_t nframes, const void *llr, int64_t llr_count, int32_t llr_type, uint8_t *out,
                     int64_t out_bytes, const vit_tuning *tune, void *workspace, size_t workspace_bytes,
                     void *stream) {
  return vit::guard_entry("vit_decode_batch", [&] {
    return decode_batch_impl(plan, codes, ncodes, frames, nframes, llr, llr_count, llr_type, out, out_bytes, tune,
                             workspace, workspace_bytes, stream);
  });
}

int vit_plan_autotune(vit_plan *plan, const vit_code *codes, int32_t ncodes, const vit_frame *frames,
                      int32_t nframes, const void *llr, int64_t llr_count, int32_t llr_type, uint8_t *out,
                      int64_t out_bytes, void *workspace, size_t workspace_bytes, void *stream, vit_tuning *chosen) {
  return vit::guard_entry("vit_plan_autotune", [&] {
    return plan_autotune_impl(plan, codes, ncodes, frames, nframes, llr, llr_count, llr_type, out, out_bytes,
                              workspace, workspace_bytes, stream, chosen);
  });
}

int vit_plan_set_tune_tolerance(vit_plan *plan, double max_diff_fraction) {
  vit::api_clear_error();
  if (!plan) return api_fail(VIT_EINVAL, "plan is NULL");
  if (!(max_diff_fraction >= 0.0 && max_diff_fraction <= 1.0))
    return api_fail(VIT_EINVAL, "tolerance %g outside [0, 1]", max_diff_fraction);
  plan->tune_tolerance = max_diff_fraction;
  return VIT_OK;
}

int vit_plan_set_metric_bits(vit_plan *plan, int32_t bits) {
  vit::api_clear_error();
  if (!plan) return api_fail(VIT_EINVAL, "plan is NULL");
  if (bits != 0 && bits != 16 && bits != 32) return api_fail(VIT_EINVAL, "metric_bits = %d (0, 16 or 32)", bits);
  plan->metric_bits = bits;
  return VIT_OK;
}

int vit_plan_get_tuning(const vit_plan *plan, vit_tuning_entry *entries, int32_t max, int32_t *count) {
  vit::api_clear_error();
  if (!plan || !count || max < 0 || (max > 0 && !entries)) return api_fail(VIT_EINVAL, "bad arguments");
  *count = (int32_t)plan->tuned.size();
  int32_t i = 0;
  for (const auto &kv : plan->tuned) {
    if (i >= max) break;
    entries[i++] = kv.second;
  }
  return VIT_OK;
}

static int plan_set_tuning_impl(vit_plan *plan, const vit_tuning_entry *entries, int32_t count) {
  vit::api_clear_error();
  if (!plan || count < 0 || (count > 0 && !entries)) return api_fail(VIT_EINVAL, "bad arguments");
  for (int32_t i = 0; i < count; ++i) {  // all entries are checked before any is taken
    const vit_tuning_entry &e = entries[i];
    int st = vit::api_check_code(&e.code);
    if (!st) st = check_tuning(e.tuning);
    if (st) {
      char why[256];
      snprintf(why, sizeof(why), "%s", vit_last_error());  // api_fail rewrites that buffer
      return api_fail(st, "entry %d: %s", i, why);
    }
    if (e.llr_type != VIT_LLR_F32 && e.llr_type != VIT_LLR_I8 && e.llr_type != VIT_LLR_HARD)
      return api_fail(VIT_EINVAL, "entry %d: unknown llr_type %d", i, e.llr_type);
    if (e.length_bucket < 0 || e.length_bucket > 40)
      return api_fail(VIT_EINVAL, "entry %d: length_bucket %d outside [0, 40]", i, e.length_bucket);
  }
  // all or nothing: the new table is built aside and swapped in
  vit::alloc_checkpoint();
  std::map<std::string, vit_tuning_entry> next = plan->tuned;
  for (int32_t i = 0; i < count; ++i) {
    vit_tuning_entry e = entries[i];
    for (int b = e.code.beta; b < 4; ++b) e.code.gen[b] = 0;
    next[tune_key(e.code, e.llr_type, e.length_bucket)] = e;
  }
  plan->tuned.swap(next);
  return VIT_OK;
}

int vit_plan_set_tuning(vit_plan *plan, const vit_tuning_entry *entries, int32_t count) {
  return vit::guard_entry("vit_plan_set_tuning", [&] { return plan_set_tuning_impl(plan, entries, count); });
}

}  // extern "C"
