// vit_server_core.h -- host-side scheduling of the serving loop, free of HIP
// so that it can be driven by a fake device in CPU tests.
//
// A request is one terminated or open frame.  The core keeps three sets:
//   pending  -- submitted, waiting for a slot and arena memory (FIFO);
//   active   -- admitted: its LLRs have arena space on the device; some of
//               its blocks are not yet launched;
//   launched -- every block launched; finishes when its last iteration does.
// An iteration admits what fits, then takes up to max_items blocks (the unit
// of Sec. III: independent once the window's LLRs are present) from the
// active frames (an equal share each, then the rest in admission order), so
// a long frame spreads over several iterations while new frames join the next
// one and can finish first.  Decoding a block needs only
// its LLR window, so between iterations a frame's device state is its arena
// range (its LLRs); path metrics live on chip for one block, and each block
// writes its decoded bytes straight to the frame's place in the host region.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <deque>
#include <vector>

namespace vit {
namespace serve {

// Ring allocator over [0, cap): allocations are taken in order; memory is
// reclaimed when the oldest live allocation is freed (frees may come in any
// order).  All sizes are multiples of `align`.
class Ring {
 public:
  explicit Ring(int64_t cap = 0, int64_t align = 256) : cap_(cap / align * align), align_(align) {}

  int64_t capacity() const { return cap_; }
  // bytes between the oldest live allocation and the next free offset
  // (includes a skipped end segment while the ring is wrapped)
  int64_t in_use() const {
    if (live_.empty()) return 0;
    const int64_t tail = live_.front().off;
    return head_ > tail ? head_ - tail : cap_ - tail + head_;
  }
  int64_t round(int64_t b) const { return (b + align_ - 1) / align_ * align_; }

  // Returns the offset, or -1 if `bytes` does not fit now.  *id receives a
  // handle for free().
  int64_t alloc(int64_t bytes, int64_t *id) {
    bytes = round(bytes > 0 ? bytes : 1);
    if (bytes > cap_) return -1;
    int64_t off;
    if (live_.empty()) {
      head_ = 0;
      off = 0;
    } else {
      const int64_t tail = live_.front().off;
      if (head_ > tail) {                     // free space: [head, cap) and [0, tail)
        if (head_ + bytes <= cap_) off = head_;
        else if (bytes <= tail) off = 0;      // wrap; [head, cap) stays unused until reclaimed
        else return -1;
      } else {                                // wrapped: free space is [head, tail)
        if (head_ + bytes <= tail) off = head_;
        else return -1;
      }
    }
    live_.push_back({off, bytes, false, next_id_});
    *id = next_id_++;
    head_ = off + bytes;
    return off;
  }

  void free(int64_t id) {
    // ids are increasing in allocation order: find by binary search
    auto it = std::lower_bound(live_.begin(), live_.end(), id,
                               [](const Entry &e, int64_t v) { return e.id < v; });
    if (it == live_.end() || it->id != id || it->freed) return;
    it->freed = true;
    while (!live_.empty() && live_.front().freed) live_.pop_front();
    if (live_.empty()) head_ = 0;
  }

  int64_t live_count() const { return (int64_t)live_.size(); }

 private:
  struct Entry {
    int64_t off, bytes;
    bool freed;
    int64_t id;
  };
  int64_t cap_, align_;
  int64_t head_ = 0;
  int64_t next_id_ = 1;
  std::deque<Entry> live_;
};

struct CodeShape {
  int k, beta;
  int64_t L, v1, v2;
};

struct Frame {
  uint64_t tag;
  int code;
  int terminated;
  int64_t n, N;
  int64_t llr_src;     // byte offset of the LLRs in the host region
  int64_t out_dst;     // byte offset of the decoded bytes in the host region
  int64_t llr_bytes;
  int64_t arrival_ns;
  // set on admission
  int64_t arena_llr = -1, ring_id = 0;
  int64_t next_cs = 0;      // first core bit not yet launched
  int64_t blocks_left = 0;  // blocks not yet launched (set on submit)
};

struct Item {          // one block: LLRs at an arena offset, output at a host-region offset
  int code;
  int64_t llr_off, out_off;
  int32_t s, e, cs, ce, flags, cost;
};

struct Copy {          // a byte range to move (ingest: host -> arena)
  int64_t src, dst, bytes;
};

constexpr int kMaxShapes = 8;

struct Iteration {
  int64_t count[kMaxShapes] = {0};  // blocks per code, handed to the sink grouped by code
  int64_t nitems = 0;
  std::vector<Copy> ingest;
  std::vector<Frame> finishing;     // frames whose last block is in this iteration
  int64_t admitted = 0;
  int64_t admit_wait_sum = 0, admit_wait_max = 0;  // admission time - arrival, ns, of its admitted frames
};

// A sink that collects the blocks into one vector, grouped by code (tests).
struct VectorSink {
  std::vector<Item> items;
  int64_t cursor[kMaxShapes] = {0};
  void begin(const int64_t *count, int ncodes) {
    int64_t total = 0;
    for (int c = 0; c < ncodes; ++c) {
      cursor[c] = total;
      total += count[c];
    }
    items.resize((size_t)total);
  }
  void put(const Item &b) { items[(size_t)cursor[b.code]++] = b; }
};

class Core {
 public:
  Core(std::vector<CodeShape> shapes, int64_t arena_bytes, int max_frames, int max_items)
      : shapes_(std::move(shapes)), ring_(arena_bytes), max_frames_(max_frames),
        max_items_(max_items) {}

  // Arena bytes a frame needs (its LLRs, 256-aligned).
  int64_t arena_need(const Frame &f) const { return ring_.round(f.llr_bytes); }
  bool fits_ever(const Frame &f) const { return arena_need(f) <= ring_.capacity(); }

  void submit(const Frame &f) {
    pending_.push_back(f);
    Frame &q = pending_.back();
    q.next_cs = 0;
    q.blocks_left = blocks_of(f);
    pending_blocks_ += q.blocks_left;
  }
  size_t pending() const { return pending_.size(); }
  // Blocks of the queued (not yet admitted) frames.
  int64_t pending_blocks() const { return pending_blocks_; }
  size_t active() const { return active_.size(); }
  int64_t frames_on_device() const { return on_device_; }
  // Frames admitted since the core was made (monotonic): the engine derives
  // its queued / on-device counts from it, so an exception part-way through
  // next_iteration leaves them consistent.
  int64_t admitted_total() const { return admitted_total_; }
  // Called by next_iteration after admission, before scheduling (the
  // server's host-allocation checkpoint, so tests can fail it there).
  void (*checkpoint)() = nullptr;
  int64_t arena_in_use() const { return ring_.in_use(); }
  bool has_work() const { return !pending_.empty() || !active_.empty(); }

  // Admit what fits, then schedule up to max_items blocks, handing each to
  // sink.put grouped by code after sink.begin(per-code counts, ncodes).
  // Returns false if there is nothing to launch (no blocks, no copies).
  // now_ns: the admission time, for the admission waits of the admitted
  // frames (0: not recorded).
  template <class Sink>
  bool next_iteration(Iteration *it, Sink &sink, int64_t now_ns = 0) {
    it->ingest.clear();
    it->finishing.clear();
    it->admitted = 0;
    it->admit_wait_sum = it->admit_wait_max = 0;
    while (!pending_.empty() && on_device_ < max_frames_) {
      Frame &f = pending_.front();
      int64_t id;
      const int64_t off = ring_.alloc(arena_need(f), &id);
      if (off < 0) break;
      f.arena_llr = off;
      f.ring_id = id;
      it->ingest.push_back({f.llr_src, f.arena_llr, f.llr_bytes});
      const int64_t w = (now_ns > 0 && now_ns > f.arrival_ns) ? now_ns - f.arrival_ns : 0;
      pending_blocks_ -= f.blocks_left;
      active_.push_back(f);
      pending_.pop_front();  // (f refers to the popped frame from here on: not used again)
      ++on_device_;
      ++admitted_total_;
      ++it->admitted;
      it->admit_wait_sum += w;
      it->admit_wait_max = w > it->admit_wait_max ? w : it->admit_wait_max;
    }
    if (checkpoint) checkpoint();
    // Blocks per frame, in two passes over the active frames in admission
    // order: first each frame gets an equal share of the iteration (at least
    // one block), so short frames that joined late finish without waiting
    // behind long ones; then what is left goes to the oldest frames.
    const size_t na = active_.size();
    take_.assign(na, 0);
    // room for every frame to finish, so that the compaction below cannot
    // throw half-way
    it->finishing.reserve(na);
    int64_t room = max_items_;
    const int64_t share = na ? std::max<int64_t>(1, room / (int64_t)na) : 0;
    for (int pass = 0; pass < 2 && room > 0; ++pass) {
      for (size_t i = 0; i < na && room > 0; ++i) {
        const int64_t left = active_[i].blocks_left - take_[i];
        const int64_t t = std::min(left, pass == 0 ? std::min(share, room) : room);
        take_[i] += t;
        room -= t;
      }
    }
    const int ncodes = (int)shapes_.size();
    for (int c = 0; c < kMaxShapes; ++c) it->count[c] = 0;
    for (size_t i = 0; i < na; ++i) it->count[active_[i].code] += take_[i];
    it->nitems = max_items_ - room;
    sink.begin(it->count, ncodes);
    // emit the blocks; frames with every block launched leave the active set
    // (one stable compaction pass: erasing from the middle one by one is
    // quadratic)
    size_t keep = 0;
    for (size_t i = 0; i < na; ++i) {
      Frame &f = active_[i];
      if (take_[i]) emit_blocks(f, take_[i], sink);
      if (f.blocks_left == 0) {
        it->finishing.push_back(f);
      } else {
        if (keep != i) active_[keep] = f;
        ++keep;
      }
    }
    active_.resize(keep);
    return it->nitems > 0 || !it->ingest.empty();
  }

  bool next_iteration(Iteration *it, VectorSink &sink, int64_t now_ns = 0) {
    return next_iteration<VectorSink>(it, sink, now_ns);
  }

  // Drop every queued and admitted frame (after a device error), reporting
  // each to fn(frame, admitted); frames of launched iterations are not
  // touched.
  template <class Fn>
  void fail_all(Fn fn) {
    for (const Frame &f : pending_) fn(f, false);
    pending_.clear();
    pending_blocks_ = 0;
    for (const Frame &f : active_) {
      fn(f, true);
      ring_.free(f.ring_id);
      --on_device_;
    }
    active_.clear();
  }

  // Queue timeouts: drop queued frames that arrived before cutoff_ns, taken
  // from the front of the queue (the order of admission) while they are
  // expired, reporting each to fn(frame).  Admitted frames always complete.
  template <class Fn>
  int64_t expire_queued(int64_t cutoff_ns, Fn fn) {
    int64_t n = 0;
    while (!pending_.empty() && pending_.front().arrival_ns < cutoff_ns) {
      fn(pending_.front());
      pending_blocks_ -= pending_.front().blocks_left;
      pending_.pop_front();
      ++n;
    }
    return n;
  }

  // The iteration has finished on the device: release its frames' arena.
  void retire(const Iteration &it) {
    for (const Frame &f : it.finishing) {
      ring_.free(f.ring_id);
      --on_device_;
    }
  }

 private:
  int64_t blocks_of(const Frame &f) const {
    const int64_t L = shapes_[f.code].L;
    return (f.n + L - 1) / L;
  }

  // Hand f's next `count` blocks (Sec. III geometry) to the sink.
  template <class Sink>
  void emit_blocks(Frame &f, int64_t count, Sink &sink) {
    const CodeShape &sh = shapes_[f.code];
    Item b;
    b.code = f.code;
    b.llr_off = f.arena_llr;
    b.out_off = f.out_dst;
    for (int64_t taken = 0; taken < count; ++taken) {
      const int64_t cs = f.next_cs;
      const int64_t ce = std::min(cs + sh.L, f.n);
      const int64_t s = std::max<int64_t>(0, cs - sh.v1);
      const int64_t e = std::min(f.N, ce + sh.v2);
      b.s = (int32_t)s;
      b.e = (int32_t)e;
      b.cs = (int32_t)cs;
      b.ce = (int32_t)ce;
      b.flags = (s == 0 ? 1 : 0) | ((f.terminated && e == f.N) ? 2 : 0);
      b.cost = (int32_t)(e - s);
      sink.put(b);
      f.next_cs = ce;
    }
    f.blocks_left -= count;
  }

  std::vector<CodeShape> shapes_;
  std::vector<int64_t> take_;
  Ring ring_;
  int max_frames_, max_items_;
  std::deque<Frame> pending_;
  std::vector<Frame> active_;  // admission order; compacted in place
  int64_t on_device_ = 0;
  int64_t admitted_total_ = 0;
  int64_t pending_blocks_ = 0;
};

}  // namespace serve
}  // namespace vit
