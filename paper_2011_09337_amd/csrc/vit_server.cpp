// vit_server.cpp -- the serving loop: continuous batching of decode requests.
//
// Requests (one frame each, LLRs in a pinned host region) are queued by
// vit_server_submit.  An engine thread owned by the server runs iterations:
// each admits queued frames while slots and device arena memory allow (the
// scheduling lives in vit_server_core.h), then issues, on the server's own
// ingest stream, one gather of the iteration's work list and of the new
// frames' LLRs from the host region into the device (over PCIe), and on the
// caller's stream, after the ingest, one batch kernel per code over the
// iteration's blocks, which write the decoded bytes straight into the host
// region, and an event.  Two iterations
// are in flight at once, so requests that arrive while the device is busy
// join the next iteration, and an iteration's ingest runs while the one
// before it decodes.
// A frame completes when the host sees its last iteration's event; its
// latency runs from its arrival time to that moment (CLOCK_MONOTONIC).
#include <hip/hip_runtime.h>
#include <string.h>
#include <time.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "vit.h"
#include "vit_guard.h"
#include "vit_internal.h"
#include "vit_shapes.h"
#include "vit_server_core.h"

namespace {

using vit::api_fail;
using vit::kHeaderBytes;
using vit::kMaxCodes;

// Iterations in flight: one decoding while the next ingests.  A third
// measured no lower latency at low load and smaller, less efficient
// iterations at high load (each iteration carries a fixed cost of about
// 0.09 ms: kernel launches and the last blocks' tails).
constexpr int kInflight = 2;
constexpr int64_t kLatSample = 1 << 24;  // latency percentiles from at most this many samples

int64_t mono_ns() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (int64_t)ts.tv_sec * 1000000000LL + ts.tv_nsec;
}

size_t round256(size_t b) { return (b + 255) / 256 * 256; }

// The header and work items go up in pieces of this many bytes, one copy
// range each, so that several workgroups of the copy kernel share them.
constexpr size_t kItemChunk = 16384;

// Device workspace per iteration slot: header | items.
size_t slot_bytes(int32_t max_items) {
  return round256(kHeaderBytes + (size_t)max_items * sizeof(vit::WorkItem));
}
size_t item_chunks(size_t bytes) { return (bytes + kItemChunk - 1) / kItemChunk; }
// Pinned staging per slot: header | items | ranges for the header and items
// and for the ingest.  The copy kernel reads the ranges in place.
size_t staging_bytes(int32_t max_frames, int32_t max_items) {
  const size_t items = slot_bytes(max_items);
  return items + (item_chunks(items) + (size_t)max_frames) * sizeof(vit::CopyRange);
}

int check_config(const vit_server_config *cfg) {
  if (!cfg) return api_fail(VIT_EINVAL, "config is NULL");
  if (cfg->size != sizeof(vit_server_config))
    return api_fail(VIT_EINVAL, "config size %u, expected %zu", cfg->size, sizeof(vit_server_config));
  if (cfg->llr_type != VIT_LLR_F32 && cfg->llr_type != VIT_LLR_I8 && cfg->llr_type != VIT_LLR_HARD)
    return api_fail(VIT_EINVAL, "unknown llr_type %d", cfg->llr_type);
  if (cfg->max_frames < 1 || cfg->max_frames > (1 << 20))
    return api_fail(VIT_EINVAL, "max_frames = %d outside [1, 2^20]", cfg->max_frames);
  if (cfg->max_items < 1 || cfg->max_items > (1 << 24))
    return api_fail(VIT_EINVAL, "max_items = %d outside [1, 2^24]", cfg->max_items);
  if (cfg->max_pending < 1) return api_fail(VIT_EINVAL, "max_pending = %d must be >= 1", cfg->max_pending);
  if (cfg->max_wait_ms < 0) return api_fail(VIT_EINVAL, "max_wait_ms = %d must be >= 0", cfg->max_wait_ms);
  if (cfg->metric_bits != 0 && cfg->metric_bits != 16 && cfg->metric_bits != 32)
    return api_fail(VIT_EINVAL, "metric_bits = %d (0, 16 or 32)", cfg->metric_bits);
  return VIT_OK;
}

bool in_range(const uint8_t *base, size_t size, const void *p, int64_t bytes) {
  const uint8_t *q = (const uint8_t *)p;
  return q >= base && bytes >= 0 && (size_t)(q - base) <= size && (size_t)bytes <= size - (size_t)(q - base);
}

// Both ends of [p, p + bytes) must be memory of the given type.
int check_memory(const void *p, size_t bytes, hipMemoryType want, const char *what) {
  hipPointerAttribute_t a0, a1;
  hipError_t e = hipPointerGetAttributes(&a0, p);
  if (e != hipSuccess) return api_fail(VIT_EINVAL, "%s: not HIP memory (%s)", what, hipGetErrorString(e));
  e = hipPointerGetAttributes(&a1, (const uint8_t *)p + bytes - 1);
  if (e != hipSuccess) return api_fail(VIT_EINVAL, "%s: its end is not HIP memory (%s)", what, hipGetErrorString(e));
  if (a0.type != want || a1.type != want)
    return api_fail(VIT_EINVAL, "%s: must be %s memory", what, want == hipMemoryTypeHost ? "pinned host" : "device");
  return VIT_OK;
}

}  // namespace

struct vit_server {
  int dev = 0;
  int num_cu = 256;
  hipStream_t stream = nullptr;
  int llr_type = VIT_LLR_I8;
  int elem = 1;
  int ncodes = 0;
  vit_code codes[kMaxCodes];
  vit_tuning shape[kMaxCodes];
  vit::BatchLaunch bl[kMaxCodes];
  uint8_t *arena = nullptr;
  size_t arena_bytes = 0;
  uint8_t *ws = nullptr;
  size_t slot_bytes = 0;
  uint8_t *host = nullptr;      // host region (host address)
  uint8_t *host_dev = nullptr;  // the same region as the device addresses it
  size_t host_bytes = 0;
  int32_t max_frames = 0, max_items = 0, max_pending = 0;
  int64_t max_wait_ns = 0;  // queue timeout, 0 = none

  void *staging[kInflight] = {};
  uint8_t *staging_dev[kInflight] = {};  // the same memory as the copy kernels address it
  hipEvent_t ev[kInflight] = {};         // the iteration is complete (its decode has written every byte)
  hipEvent_t ingested[kInflight] = {};   // its work list and LLRs are on the device
  hipEvent_t t_ingest[kInflight] = {};   // its ingest starts (timing)
  hipEvent_t t_decode[kInflight] = {};   // its decode starts (timing)
  hipStream_t ingest = nullptr;          // the server's own stream for the ingest

  // Shared with the callers, under `mu`: the hand-off queue, completions,
  // counters.  The lock is never held while a work list is built or HIP is
  // called.
  std::mutex mu;
  std::condition_variable cv;      // wakes the engine: submit, stop
  std::condition_variable idle_cv; // wakes drain: progress
  std::vector<vit::serve::Frame> incoming;
  std::deque<vit_completion> done;
  std::vector<int64_t> lat;        // latencies: all, or a uniform sample of kLatSample once more arrive
  int64_t lat_seen = 0, lat_max = 0;
  uint64_t lat_rng = 0x9e3779b97f4a7c15ull;
  int64_t submitted = 0, completed = 0, failed_frames = 0, bits_completed = 0, iterations = 0,
          items_launched = 0, peak_arena = 0, peak_frames = 0, first_arrival = 0, last_done = 0;
  int64_t iter_ingest = 0, iter_decode = 0, iter_max = 0, admit_wait = 0, admit_wait_max = 0, submit_lag = 0,
          submit_lag_max = 0, submit_lag_count = 0, engine_host = 0;
  int64_t waiting = 0;             // submitted, not yet admitted
  int64_t on_device = 0;           // admitted, not yet finished
  int status = VIT_OK;
  std::string fail_msg;
  bool stop = false;

  // Private to the engine thread.
  vit::serve::Core *core = nullptr;
  vit::serve::Iteration iters[kInflight];  // reused, so their buffers keep their capacity
  std::deque<int> inflight;                // slots of the iterations on the device, oldest first
  int next_slot = 0;
  int64_t admitted_seen = 0;               // core admissions already moved from `waiting` to `on_device`
  std::thread engine;
};

namespace {

// Writes the iteration's blocks straight into the slot's pinned staging, as
// the batch kernels read them: one run per code after the header.
struct StagingSink {
  vit::WorkItem *wi;
  int64_t cursor[kMaxCodes];
  void begin(const int64_t *count, int ncodes) {
    int64_t off = 0;
    for (int c = 0; c < ncodes; ++c) {
      cursor[c] = off;
      off += count[c];
    }
  }
  void put(const vit::serve::Item &b) {
    vit::WorkItem &w = wi[cursor[b.code]++];
    w.llr_off = b.llr_off;
    w.out_off = b.out_off;
    w.s = b.s;
    w.e = b.e;
    w.cs = b.cs;
    w.ce = b.ce;
    w.flags = b.flags;
    w.cost = b.cost;
  }
};

// Complete the slot's staging (header, copy ranges after the blocks) and
// issue the iteration's work.  Called by the engine thread without the lock.
int launch_iteration(vit_server *s, const vit::serve::Iteration &it, int slot, std::string *msg) {
  uint8_t *stg = (uint8_t *)s->staging[slot];
  uint8_t *wsd = s->ws + (size_t)slot * s->slot_bytes;
  int32_t *header = (int32_t *)stg;
  memset(header, 0, kHeaderBytes);
  int64_t off = 0;
  for (int c = 0; c < s->ncodes; ++c) {
    header[kMaxCodes + c] = (int32_t)it.count[c];
    header[2 * kMaxCodes + c] = (int32_t)off;
    off += it.count[c];
  }
  // ranges (in the staging, after the largest item list): the header and
  // items in pieces, then the admitted frames' LLRs
  const size_t items_end = kHeaderBytes + (size_t)it.nitems * sizeof(vit::WorkItem);
  const size_t ranges_at = slot_bytes(s->max_items);
  vit::CopyRange *cr = (vit::CopyRange *)(stg + ranges_at);
  const size_t nchunk = item_chunks(items_end);
  for (size_t i = 0; i < nchunk; ++i) {
    const size_t at = i * kItemChunk;
    cr[i] = {s->staging_dev[slot] + at, wsd + at, (int64_t)std::min(kItemChunk, items_end - at), 0};
  }
  vit::CopyRange *ir = cr + nchunk;
  for (size_t i = 0; i < it.ingest.size(); ++i)
    ir[i] = {s->host_dev + it.ingest[i].src, s->arena + it.ingest[i].dst, it.ingest[i].bytes, 0};
  const vit::CopyRange *dcr = (const vit::CopyRange *)(s->staging_dev[slot] + ranges_at);

  // ingest on the server's stream: one copy kernel gathers the work list and
  // the new frames' LLRs from pinned host memory, reading its ranges there
  // (no separate upload of the staging); it overlaps the decode of the
  // iteration before, whose arena ranges and workspace slot it does not
  // touch: slots are reused only after their iteration retired, and the
  // ring allocator gives new frames free arena
  hipError_t e = hipEventRecord(s->t_ingest[slot], s->ingest);
  if (e != hipSuccess) return *msg = std::string("hipEventRecord: ") + hipGetErrorString(e), VIT_EDEVICE;
  e = vit::launch_copy_list(dcr, (int32_t)(nchunk + it.ingest.size()), s->ingest);
  if (e != hipSuccess) return *msg = std::string("ingest: ") + hipGetErrorString(e), VIT_EDEVICE;
  e = hipEventRecord(s->ingested[slot], s->ingest);
  if (e != hipSuccess) return *msg = std::string("hipEventRecord: ") + hipGetErrorString(e), VIT_EDEVICE;
  e = hipStreamWaitEvent(s->stream, s->ingested[slot], 0);
  if (e != hipSuccess) return *msg = std::string("hipStreamWaitEvent: ") + hipGetErrorString(e), VIT_EDEVICE;
  e = hipEventRecord(s->t_decode[slot], s->stream);
  if (e != hipSuccess) return *msg = std::string("hipEventRecord: ") + hipGetErrorString(e), VIT_EDEVICE;
  for (int c = 0; c < s->ncodes; ++c) {
    if (!it.count[c]) continue;
    vit::BatchArgs a;
    a.llr = s->arena;
    a.out = s->host_dev;  // items carry each frame's output offset in the host region
    a.header = (int32_t *)wsd;
    a.items = (const vit::WorkItem *)(wsd + kHeaderBytes);
    a.code_index = c;
    for (int b = 0; b < 4; ++b) a.gen[b] = b < s->codes[c].beta ? s->codes[c].gen[b] : 0u;
    int words = s->bl[c].lds_words_per_wave;
    void *kargs[] = {&a, &words};
    const unsigned grid =
        vit::batch_launch_grid(s->bl[c], it.count[c], (int64_t)s->shape[c].L + s->shape[c].v, s->num_cu);
    e = hipLaunchKernel(s->bl[c].fn, dim3(grid), dim3(s->bl[c].block), kargs, s->bl[c].lds, s->stream);
    if (e != hipSuccess) return *msg = std::string("decode launch: ") + hipGetErrorString(e), VIT_EDEVICE;
  }
  e = hipEventRecord(s->ev[slot], s->stream);
  if (e != hipSuccess) return *msg = std::string("hipEventRecord: ") + hipGetErrorString(e), VIT_EDEVICE;
  return VIT_OK;
}

void fail_locked(vit_server *s, int status, const std::string &msg) {
  if (s->status == VIT_OK) {
    s->status = status;
    s->fail_msg = msg;
  }
}

// Move the core's new admissions from the queued count to the on-device
// count (engine thread).
void sync_admitted(vit_server *s) {
  const int64_t total = s->core->admitted_total();
  if (total == s->admitted_seen) return;
  std::lock_guard<std::mutex> lk(s->mu);
  s->waiting -= total - s->admitted_seen;
  s->on_device += total - s->admitted_seen;
  s->admitted_seen = total;
}

// Report finished (or failed) frames; `admitted` of them were on the device,
// the rest were still waiting.  The counts drop first, so that an allocation
// failure while the completions are queued loses completions, never the
// server's accounting (drain still returns).
void finish_frames(vit_server *s, const std::vector<vit::serve::Frame> &frames, int st, int64_t now,
                   int64_t admitted) {
  std::lock_guard<std::mutex> lk(s->mu);
  s->on_device -= admitted;
  s->waiting -= (int64_t)frames.size() - admitted;
  s->last_done = now;
  s->idle_cv.notify_all();
  for (const auto &f : frames) {
    s->done.push_back({f.tag, st, 0, f.arrival_ns, now});
    if (st == VIT_OK) {
      ++s->completed;
      s->bits_completed += f.n;
      // reservoir sampling keeps the percentiles' memory bounded
      const int64_t l = now - f.arrival_ns;
      if ((int64_t)s->lat.size() < kLatSample) {
        s->lat.push_back(l);
      } else {
        s->lat_rng ^= s->lat_rng << 13;
        s->lat_rng ^= s->lat_rng >> 7;
        s->lat_rng ^= s->lat_rng << 17;
        const uint64_t r = s->lat_rng % (uint64_t)(s->lat_seen + 1);
        if (r < (uint64_t)kLatSample) s->lat[r] = l;
      }
      ++s->lat_seen;
      s->lat_max = std::max(s->lat_max, l);
    } else {
      ++s->failed_frames;
    }
  }
}

void engine_loop(vit_server *s) {
  std::vector<vit::serve::Frame> arrived;
  std::vector<vit::serve::Frame> expired;
  std::vector<vit::serve::Frame> dropped;
  for (;;) {
    bool stop, failed;
    {
      std::lock_guard<std::mutex> lk(s->mu);
      arrived.swap(s->incoming);
      stop = s->stop;
      failed = s->status != VIT_OK;
    }
    for (const auto &f : arrived) s->core->submit(f);
    arrived.clear();
    sync_admitted(s);  // also catches up after an exception inside next_iteration
    if (s->max_wait_ns > 0 && !failed) {
      // queue timeouts, before anything more is admitted
      const int64_t now = mono_ns();
      expired.clear();
      s->core->expire_queued(now - s->max_wait_ns, [&](const vit::serve::Frame &f) { expired.push_back(f); });
      if (!expired.empty()) finish_frames(s, expired, VIT_ETIMEDOUT, now, 0);
    }

    // retire finished iterations, oldest first
    bool progressed = false;
    while (!s->inflight.empty()) {
      const hipError_t q = hipEventQuery(s->ev[s->inflight.front()]);
      if (q == hipErrorNotReady) break;
      const int st = q == hipSuccess ? VIT_OK : VIT_EDEVICE;
      if (st != VIT_OK) {
        std::lock_guard<std::mutex> lk(s->mu);
        fail_locked(s, st, std::string("iteration failed: ") + hipGetErrorString(q));
        failed = true;
      }
      // leave the in-flight list before reporting, so that a failure while
      // reporting cannot report the iteration twice
      const int slot = s->inflight.front();
      vit::serve::Iteration &it = s->iters[slot];
      s->inflight.pop_front();
      if (st == VIT_OK) {
        float a = 0, b = 0, c = 0;
        if (hipEventElapsedTime(&a, s->t_ingest[slot], s->ingested[slot]) == hipSuccess &&
            hipEventElapsedTime(&b, s->t_decode[slot], s->ev[slot]) == hipSuccess &&
            hipEventElapsedTime(&c, s->t_ingest[slot], s->ev[slot]) == hipSuccess) {
          std::lock_guard<std::mutex> lk(s->mu);
          s->iter_ingest += (int64_t)(a * 1e6f);
          s->iter_decode += (int64_t)(b * 1e6f);
          s->iter_max = std::max(s->iter_max, (int64_t)(c * 1e6f));
        }
      }
      s->core->retire(it);
      progressed = true;
      finish_frames(s, it.finishing, st, mono_ns(), (int64_t)it.finishing.size());
    }
    if (failed && s->inflight.empty() && s->core->has_work()) {
      // after a device error nothing more is launched: queued and admitted
      // frames complete with the error
      dropped.clear();
      int64_t admitted = 0;
      s->core->fail_all([&](const vit::serve::Frame &f, bool adm) {
        dropped.push_back(f);
        admitted += adm ? 1 : 0;
      });
      int st;
      {
        std::lock_guard<std::mutex> lk(s->mu);
        st = s->status;
      }
      finish_frames(s, dropped, st, mono_ns(), admitted);
    }
    if (stop && s->inflight.empty()) break;
    // Launch policy: a new iteration goes out when a slot is free and the
    // newest iteration in flight has finished its ingest (it is decoding or
    // waiting to decode).  Work that arrives during an ingest then joins the
    // next iteration instead of a small one of its own: every iteration
    // carries a fixed device cost (launches, the last blocks' tails), so
    // fewer, larger iterations carry more at high load, while at low load the
    // ingests are short and the wait is too.  When the queue already holds
    // more blocks than an iteration takes, waiting cannot make the next one
    // larger: it is built at once, so that the host's work on it overlaps
    // the ingest in flight.
    bool slot_free = (int)s->inflight.size() < kInflight;
    bool deferred = false;
    if (slot_free && !s->inflight.empty() && s->core->has_work() && s->core->pending_blocks() < s->max_items) {
      if (hipEventQuery(s->ingested[s->inflight.back()]) == hipErrorNotReady) {
        slot_free = false;
        deferred = true;
      }
    }
    if (!failed && !stop && slot_free && s->core->has_work()) {
      const int64_t t_host = mono_ns();
      const int slot = s->next_slot;
      vit::serve::Iteration &it = s->iters[slot];
      StagingSink sink;
      sink.wi = (vit::WorkItem *)((uint8_t *)s->staging[slot] + kHeaderBytes);
      const bool any = s->core->next_iteration(&it, sink, mono_ns());
      sync_admitted(s);
      if (any) {
        s->next_slot = (slot + 1) % kInflight;
        {
          std::lock_guard<std::mutex> lk(s->mu);
          s->admit_wait += it.admit_wait_sum;
          s->admit_wait_max = std::max(s->admit_wait_max, it.admit_wait_max);
          s->peak_arena = std::max(s->peak_arena, s->core->arena_in_use());
          s->peak_frames = std::max(s->peak_frames, s->core->frames_on_device());
          ++s->iterations;
          s->items_launched += it.nitems;
        }
        s->inflight.push_back(slot);
        std::string msg;
        const int st = launch_iteration(s, it, slot, &msg);
        {
          std::lock_guard<std::mutex> lk(s->mu);
          s->engine_host += mono_ns() - t_host;
        }
        if (st != VIT_OK) {
          {
            std::lock_guard<std::mutex> lk(s->mu);
            fail_locked(s, st, msg);
          }
          // the iteration's event was not recorded: its frames fail now
          s->inflight.pop_back();
          s->core->retire(it);
          finish_frames(s, it.finishing, st, mono_ns(), (int64_t)it.finishing.size());
        }
        continue;
      }
    }
    if (progressed) continue;
    // nothing to launch now: wait for a submit, or poll the running
    // iterations (a deferred launch polls without waiting for submits, which
    // cannot make it go out sooner)
    std::unique_lock<std::mutex> lk(s->mu);
    if (deferred) {
      if (!s->stop) s->cv.wait_for(lk, std::chrono::microseconds(10), [&] { return s->stop; });
      continue;
    }
    if (!s->incoming.empty() || s->stop) continue;
    if (!s->inflight.empty()) s->cv.wait_for(lk, std::chrono::microseconds(20));
    else s->cv.wait_for(lk, std::chrono::milliseconds(2));
  }
}

// The engine thread.  A host allocation failure inside the loop fails the
// server with VIT_ENOMEM and the loop resumes in its failed mode: running
// iterations retire and the frames still queued complete with the error (a
// frame that was being handed over when the allocation failed may be lost).
void engine_main(vit_server *s) {
  (void)hipSetDevice(s->dev);
  for (;;) {
    try {
      engine_loop(s);
      return;
    } catch (const std::exception &e) {
      std::lock_guard<std::mutex> lk(s->mu);
      fail_locked(s, VIT_ENOMEM, std::string("engine: ") + e.what());
    } catch (...) {
      std::lock_guard<std::mutex> lk(s->mu);
      fail_locked(s, VIT_ENOMEM, "engine: host resource failure");
    }
    // if allocations keep failing, do not spin on them
    std::this_thread::sleep_for(std::chrono::milliseconds(1));
  }
}

}  // namespace

extern "C" {

int vit_server_workspace_size(const vit_server_config *cfg, size_t *bytes) {
  vit::api_clear_error();
  int st = check_config(cfg);
  if (st) return st;
  if (!bytes) return api_fail(VIT_EINVAL, "bytes is NULL");
  *bytes = kInflight * slot_bytes(cfg->max_items);
  return VIT_OK;
}

static int server_create_impl(const vit_code *codes, int32_t ncodes, const vit_tuning *tune,
                              const vit_server_config *cfg, vit_server **out) {
  vit::api_clear_error();
  if (!out) return api_fail(VIT_EINVAL, "server is NULL");
  *out = nullptr;
  if (!codes || ncodes < 1 || ncodes > kMaxCodes) return api_fail(VIT_EINVAL, "ncodes = %d outside [1, 8]", ncodes);
  int st;
  for (int c = 0; c < ncodes; ++c)
    if ((st = vit::api_check_code(&codes[c]))) return st;
  if ((st = check_config(cfg))) return st;
  vit_tuning shape[kMaxCodes];
  for (int c = 0; c < ncodes; ++c) {
    if (tune) {
      shape[c] = tune[c];
    } else {
      shape[c].L = 256;
      shape[c].v = vit::default_overlap(codes[c].k);
      shape[c].v1 = -1;
      shape[c].waves_per_block = 1;
    }
    const vit_tuning &t = shape[c];
    if (t.L <= 0 || t.L % 8 != 0) return api_fail(VIT_EINVAL, "code %d: L = %d must be a positive multiple of 8", c, t.L);
    if (t.v < 0 || t.v1 < -1 || t.v1 > t.v) return api_fail(VIT_EINVAL, "code %d: bad overlap (v %d, v1 %d)", c, t.v, t.v1);
    if (t.waves_per_block < 1 || t.waves_per_block > 4)
      return api_fail(VIT_EINVAL, "code %d: waves_per_block = %d outside [1, 4]", c, t.waves_per_block);
    st = vit::integer_shape_precheck(codes[c].k, codes[c].beta, cfg->llr_type, cfg->metric_bits, (int64_t)t.L + t.v,
                                     false);
    if (st) return st;
  }
  if (!cfg->arena || !cfg->workspace || !cfg->host) return api_fail(VIT_EINVAL, "NULL arena, workspace or host region");
  if ((((uintptr_t)cfg->arena | (uintptr_t)cfg->workspace) & 255u) != 0)
    return api_fail(VIT_EINVAL, "arena and workspace must be 256-byte aligned");
  const size_t need_ws = kInflight * slot_bytes(cfg->max_items);
  if (cfg->workspace_bytes < need_ws)
    return api_fail(VIT_EINVAL, "workspace of %zu bytes, %zu needed", cfg->workspace_bytes, need_ws);
  if (cfg->arena_bytes < 256 || cfg->host_bytes < 1) return api_fail(VIT_EINVAL, "empty arena or host region");

  // from here on the device is used
  if ((st = check_memory(cfg->arena, cfg->arena_bytes, hipMemoryTypeDevice, "arena"))) return st;
  if ((st = check_memory(cfg->workspace, cfg->workspace_bytes, hipMemoryTypeDevice, "workspace"))) return st;
  if ((st = check_memory(cfg->host, cfg->host_bytes, hipMemoryTypeHost, "host region"))) return st;

  vit_server *s = vit::alloc_checkpoint_fails() ? nullptr : new (std::nothrow) vit_server();
  if (!s) return api_fail(VIT_ENOMEM, "server allocation failed");
  auto bail = [&](int status) {
    for (int i = 0; i < kInflight; ++i) {
      if (s->staging[i]) (void)hipHostFree(s->staging[i]);
      if (s->ev[i]) (void)hipEventDestroy(s->ev[i]);
      if (s->ingested[i]) (void)hipEventDestroy(s->ingested[i]);
      if (s->t_ingest[i]) (void)hipEventDestroy(s->t_ingest[i]);
      if (s->t_decode[i]) (void)hipEventDestroy(s->t_decode[i]);
    }
    if (s->ingest) (void)hipStreamDestroy(s->ingest);
    delete s->core;
    delete s;
    return status;
  };
  hipError_t e = hipGetDevice(&s->dev);
  if (e != hipSuccess) return bail(vit::api_fail_hip(e, "hipGetDevice"));
  e = hipDeviceGetAttribute(&s->num_cu, hipDeviceAttributeMultiprocessorCount, s->dev);
  if (e != hipSuccess) return bail(vit::api_fail_hip(e, "hipDeviceGetAttribute"));
  void *hd = nullptr;
  e = hipHostGetDevicePointer(&hd, cfg->host, 0);
  if (e != hipSuccess) return bail(vit::api_fail_hip(e, "hipHostGetDevicePointer"));
  s->stream = (hipStream_t)cfg->stream;
  s->llr_type = cfg->llr_type;
  s->elem = cfg->llr_type == VIT_LLR_F32 ? 4 : 1;
  s->ncodes = ncodes;
  s->arena = (uint8_t *)cfg->arena;
  s->arena_bytes = cfg->arena_bytes;
  s->ws = (uint8_t *)cfg->workspace;
  s->slot_bytes = slot_bytes(cfg->max_items);
  s->host = (uint8_t *)cfg->host;
  s->host_dev = (uint8_t *)hd;
  s->host_bytes = cfg->host_bytes;
  s->max_frames = cfg->max_frames;
  s->max_items = cfg->max_items;
  s->max_pending = cfg->max_pending;
  s->max_wait_ns = (int64_t)cfg->max_wait_ms * 1000000;
  std::vector<vit::serve::CodeShape> shapes;
  try {
    shapes.reserve((size_t)ncodes);
  } catch (const std::bad_alloc &) {
    return bail(api_fail(VIT_ENOMEM, "shape list allocation failed"));
  }
  for (int c = 0; c < ncodes; ++c) {
    s->codes[c] = codes[c];
    s->shape[c] = shape[c];
    int unsupported = 0;
    const char *why = "";
    e = vit::plan_batch_launch(codes[c].k, codes[c].beta, codes[c].gen, cfg->llr_type, cfg->metric_bits,
                               (int64_t)shape[c].L + shape[c].v, shape[c].waves_per_block, &s->bl[c], &unsupported,
                               &why);
    if (e != hipSuccess) return bail(vit::api_fail_hip(e, "batch launch planning"));
    if (unsupported) return bail(api_fail(VIT_EUNSUPPORTED, "code %d: %s", c, why));
    const int64_t v1 = shape[c].v1 < 0 ? shape[c].v / 2 : shape[c].v1;
    shapes.push_back({codes[c].k, codes[c].beta, shape[c].L, v1, shape[c].v - v1});
  }
  for (int i = 0; i < kInflight; ++i) {
    // coherent: the copy kernels read the ranges and items in place, and
    // the host rewrites the slot every other iteration
    e = hipHostMalloc(&s->staging[i], staging_bytes(cfg->max_frames, cfg->max_items),
                      hipHostMallocMapped | hipHostMallocCoherent);
    if (e != hipSuccess) return bail(vit::api_fail_hip(e, "hipHostMalloc"));
    void *sd = nullptr;
    e = hipHostGetDevicePointer(&sd, s->staging[i], 0);
    if (e != hipSuccess) return bail(vit::api_fail_hip(e, "hipHostGetDevicePointer"));
    s->staging_dev[i] = (uint8_t *)sd;
    // timing events: the statistics report the device time of each iteration
    e = hipEventCreate(&s->ev[i]);
    if (e != hipSuccess) return bail(vit::api_fail_hip(e, "hipEventCreate"));
    e = hipEventCreate(&s->ingested[i]);
    if (e != hipSuccess) return bail(vit::api_fail_hip(e, "hipEventCreate"));
    e = hipEventCreate(&s->t_ingest[i]);
    if (e != hipSuccess) return bail(vit::api_fail_hip(e, "hipEventCreate"));
    e = hipEventCreate(&s->t_decode[i]);
    if (e != hipSuccess) return bail(vit::api_fail_hip(e, "hipEventCreate"));
  }
  // default priority, like every stream of the library
  e = hipStreamCreateWithFlags(&s->ingest, hipStreamNonBlocking);
  if (e != hipSuccess) return bail(vit::api_fail_hip(e, "hipStreamCreate"));
  try {
    vit::alloc_checkpoint();
    s->core = new vit::serve::Core(shapes, (int64_t)cfg->arena_bytes, cfg->max_frames, cfg->max_items);
    s->core->checkpoint = &vit::alloc_checkpoint;
  } catch (const std::bad_alloc &) {
    return bail(api_fail(VIT_ENOMEM, "core allocation failed"));
  }
  try {
    s->engine = std::thread(engine_main, s);
  } catch (...) {
    return bail(api_fail(VIT_ENOMEM, "could not start the engine thread"));
  }
  *out = s;
  return VIT_OK;
}

static int server_submit_impl(vit_server *s, const vit_request *reqs, int32_t count, int32_t *accepted) {
  vit::api_clear_error();
  if (accepted) *accepted = 0;
  if (!s) return api_fail(VIT_EINVAL, "server is NULL");
  if (count < 0 || (count > 0 && !reqs)) return api_fail(VIT_EINVAL, "bad request array");
  const int64_t now = mono_ns();
  // validate outside the lock (only immutable server state is read)
  thread_local std::vector<vit::serve::Frame> local;
  local.clear();
  int st = VIT_OK;
  for (int32_t i = 0; i < count; ++i) {
    const vit_request &r = reqs[i];
    if (r.code_id < 0 || r.code_id >= s->ncodes) {
      st = api_fail(VIT_EINVAL, "request %d: code_id %d", i, r.code_id);
      break;
    }
    if (r.n <= 0 || (r.terminated != 0 && r.terminated != 1)) {
      st = api_fail(VIT_EINVAL, "request %d: n = %lld, terminated = %d", i, (long long)r.n, r.terminated);
      break;
    }
    const vit_code &c = s->codes[r.code_id];
    const int64_t N = r.n + (r.terminated ? c.k - 1 : 0);
    if (N * c.beta * s->elem >= ((int64_t)1 << 31)) {
      st = api_fail(VIT_EUNSUPPORTED, "request %d: frame too long", i);
      break;
    }
    vit::serve::Frame f;
    f.tag = r.tag;
    f.code = r.code_id;
    f.terminated = r.terminated;
    f.n = r.n;
    f.N = N;
    f.llr_bytes = N * c.beta * s->elem;
    if (!in_range(s->host, s->host_bytes, r.llr, f.llr_bytes) ||
        !in_range(s->host, s->host_bytes, r.out, (r.n + 7) / 8)) {
      st = api_fail(VIT_EINVAL, "request %d: LLRs or output outside the host region", i);
      break;
    }
    f.llr_src = (const uint8_t *)r.llr - s->host;
    f.out_dst = r.out - s->host;
    f.arrival_ns = r.arrival_ns > 0 ? r.arrival_ns : now;
    if (!s->core->fits_ever(f)) {  // reads only the arena size, fixed at creation
      st = api_fail(VIT_EINVAL, "request %d: needs %lld arena bytes, more than the arena", i,
                    (long long)s->core->arena_need(f));
      break;
    }
    local.push_back(f);
  }
  int32_t took = (int32_t)local.size();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->status != VIT_OK) return api_fail(s->status, "server failed: %s", s->fail_msg.c_str());
    const int64_t room = std::max<int64_t>(0, (int64_t)s->max_pending - s->waiting);
    if (took > room) {
      took = (int32_t)room;
      st = api_fail(VIT_EBUSY, "request queue full (%d waiting)", s->max_pending);
    }
    s->incoming.reserve(s->incoming.size() + (size_t)took);  // may throw: nothing is queued yet
    s->incoming.insert(s->incoming.end(), local.begin(), local.begin() + took);
    s->waiting += took;
    s->submitted += took;
    for (int32_t i = 0; i < took; ++i) {
      if (s->first_arrival == 0 || local[i].arrival_ns < s->first_arrival) s->first_arrival = local[i].arrival_ns;
      if (reqs[i].arrival_ns > 0) {  // a stated arrival time: how late it is handed over
        const int64_t lag = now > reqs[i].arrival_ns ? now - reqs[i].arrival_ns : 0;
        s->submit_lag += lag;
        s->submit_lag_max = std::max(s->submit_lag_max, lag);
        ++s->submit_lag_count;
      }
    }
  }
  if (took) s->cv.notify_one();
  if (accepted) *accepted = took;
  return st;
}

int vit_server_submit_paced(vit_server *s, const vit_request *reqs, int32_t count, int32_t *accepted) {
  vit::api_clear_error();
  if (accepted) *accepted = 0;
  if (!s) return api_fail(VIT_EINVAL, "server is NULL");
  if (count < 0 || (count > 0 && !reqs)) return api_fail(VIT_EINVAL, "bad request array");
  int32_t i = 0;
  while (i < count) {
    const int64_t now = mono_ns();
    int32_t j = i;
    while (j < count && reqs[j].arrival_ns <= now) ++j;
    if (j > i) {
      int32_t took = 0;
      const int st = vit_server_submit(s, reqs + i, j - i, &took);
      i += took;
      if (accepted) *accepted = i;
      if (st == VIT_EBUSY) {
        std::this_thread::sleep_for(std::chrono::microseconds(50));
        continue;
      }
      if (st != VIT_OK) return st;
      continue;
    }
    const int64_t wait = reqs[i].arrival_ns - now;
    if (wait > 300000) std::this_thread::sleep_for(std::chrono::nanoseconds(wait - 200000));
    else if (wait > 20000) std::this_thread::yield();
  }
  return VIT_OK;
}

int vit_server_poll(vit_server *s, vit_completion *out, int32_t max, int32_t *count) {
  vit::api_clear_error();
  if (count) *count = 0;
  if (!s || !count || max < 0 || (max > 0 && !out)) return api_fail(VIT_EINVAL, "bad poll arguments");
  std::lock_guard<std::mutex> lk(s->mu);
  int32_t n = 0;
  while (n < max && !s->done.empty()) {
    out[n++] = s->done.front();
    s->done.pop_front();
  }
  *count = n;
  return VIT_OK;
}

int vit_server_drain(vit_server *s, int64_t timeout_ms) {
  vit::api_clear_error();
  if (!s) return api_fail(VIT_EINVAL, "server is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  auto idle = [&] { return s->waiting == 0 && s->on_device == 0; };
  if (timeout_ms < 0) {
    s->idle_cv.wait(lk, idle);
  } else if (!s->idle_cv.wait_for(lk, std::chrono::milliseconds(timeout_ms), idle)) {
    return api_fail(VIT_EBUSY, "work still queued after %lld ms", (long long)timeout_ms);
  }
  if (s->status != VIT_OK) return api_fail(s->status, "server failed: %s", s->fail_msg.c_str());
  return VIT_OK;
}

static int server_stats_impl(vit_server *s, vit_serve_stats *st, int32_t reset) {
  vit::api_clear_error();
  if (!s || !st) return api_fail(VIT_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  memset(st, 0, sizeof(*st));
  st->submitted = s->submitted;
  st->completed = s->completed;
  st->failed = s->failed_frames;
  st->bits_completed = s->bits_completed;
  st->iterations = s->iterations;
  st->items_launched = s->items_launched;
  st->pending = s->waiting;
  st->frames_on_device = s->on_device;
  st->peak_frames_on_device = s->peak_frames;
  st->peak_arena_bytes = s->peak_arena;
  st->first_arrival_ns = s->first_arrival;
  st->last_done_ns = s->last_done;
  st->iter_ingest_ns = s->iter_ingest;
  st->iter_decode_ns = s->iter_decode;
  st->iter_max_ns = s->iter_max;
  st->admit_wait_ns = s->admit_wait;
  st->admit_wait_max_ns = s->admit_wait_max;
  st->submit_lag_ns = s->submit_lag;
  st->submit_lag_max_ns = s->submit_lag_max;
  st->submit_lag_count = s->submit_lag_count;
  st->engine_host_ns = s->engine_host;
  if (!s->lat.empty()) {
    vit::alloc_checkpoint();
    std::vector<int64_t> v(s->lat);
    auto pct = [&](double p) {
      size_t i = (size_t)(p * (double)(v.size() - 1) + 0.5);
      std::nth_element(v.begin(), v.begin() + (std::ptrdiff_t)i, v.end());
      return v[i];
    };
    st->p50_ns = pct(0.50);
    st->p99_ns = pct(0.99);
    st->max_ns = s->lat_max;
  }
  if (reset) {
    s->lat.clear();
    s->lat_seen = 0;
    s->lat_max = 0;
    s->submitted = s->completed = s->failed_frames = s->bits_completed = 0;
    s->iterations = s->items_launched = 0;
    s->peak_arena = s->peak_frames = 0;
    s->first_arrival = s->last_done = 0;
    s->iter_ingest = s->iter_decode = s->iter_max = 0;
    s->admit_wait = s->admit_wait_max = 0;
    s->submit_lag = s->submit_lag_max = s->submit_lag_count = 0;
    s->engine_host = 0;
  }
  return VIT_OK;
}

void vit_server_destroy(vit_server *s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  if (s->engine.joinable()) s->engine.join();
  // every iteration has retired, so its ingest (which its decode waited
  // for) is complete too
  for (int i = 0; i < kInflight; ++i) {
    if (s->staging[i]) (void)hipHostFree(s->staging[i]);
    if (s->ev[i]) (void)hipEventDestroy(s->ev[i]);
    if (s->ingested[i]) (void)hipEventDestroy(s->ingested[i]);
    if (s->t_ingest[i]) (void)hipEventDestroy(s->t_ingest[i]);
    if (s->t_decode[i]) (void)hipEventDestroy(s->t_decode[i]);
  }
  if (s->ingest) (void)hipStreamDestroy(s->ingest);
  delete s->core;
  delete s;
}

// The entry points that allocate: no exception leaves the C ABI (vit_guard.h).
int vit_server_create(const vit_code *codes, int32_t ncodes, const vit_tuning *tune, const vit_server_config *cfg,
                      vit_server **out) {
  return vit::guard_entry("vit_server_create", [&] { return server_create_impl(codes, ncodes, tune, cfg, out); });
}

int vit_server_submit(vit_server *s, const vit_request *reqs, int32_t count, int32_t *accepted) {
  return vit::guard_entry("vit_server_submit", [&] { return server_submit_impl(s, reqs, count, accepted); });
}

int vit_server_stats(vit_server *s, vit_serve_stats *st, int32_t reset) {
  return vit::guard_entry("vit_server_stats", [&] { return server_stats_impl(s, st, reset); });
}

}  // extern "C"
