// Host-only check of the serving loop's scheduler (vit_server_core.h) against
// a fake device: iterations "run" in launch order and finish at random
// moments.  Every invariant the HIP engine relies on is asserted here:
// block geometry per frame (blocked decoding with overlap), each core bit
// launched exactly once and in order, ingest no later than a frame's first
// block, completion in the iteration of its last block, items writing to the
// frame's own output place, arena ranges of frames on
// the device pairwise disjoint and inside the arena, slot and item limits,
// FIFO admission, a block for every waiting frame when the iteration has room
// for one each, and eventual completion.
//
// usage: server_core_check SEED
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <deque>
#include <map>
#include <random>
#include <set>
#include <vector>

#include "vit_server_core.h"

using namespace vit::serve;

#define CHECK(c, ...)                                   \
  do {                                                  \
    if (!(c)) {                                         \
      fprintf(stderr, "FAIL line %d: ", __LINE__);      \
      fprintf(stderr, __VA_ARGS__);                     \
      fprintf(stderr, "\n");                            \
      exit(1);                                          \
    }                                                   \
  } while (0)

static void ring_check(std::mt19937_64 &rng) {
  const int64_t cap = 256 * (1 + (int64_t)(rng() % 64));
  Ring r(cap);
  struct Live { int64_t off, bytes, id; };
  std::vector<Live> live;
  for (int step = 0; step < 20000; ++step) {
    if (live.empty() || rng() % 3 != 0) {
      const int64_t want = 1 + (int64_t)(rng() % (uint64_t)(cap / 3 + 1));
      int64_t id;
      const int64_t off = r.alloc(want, &id);
      if (live.empty()) CHECK(off == 0 || want > cap, "empty ring refused %lld of %lld", (long long)want, (long long)cap);
      if (off >= 0) {
        const int64_t b = r.round(want);
        CHECK(off % 256 == 0 && off + b <= cap, "allocation [%lld, +%lld) outside the ring", (long long)off, (long long)b);
        for (const Live &l : live)
          CHECK(off + b <= l.off || l.off + l.bytes <= off, "overlap [%lld,+%lld) with [%lld,+%lld)", (long long)off,
                (long long)b, (long long)l.off, (long long)l.bytes);
        live.push_back({off, b, id});
      }
    } else {
      const size_t i = rng() % live.size();
      r.free(live[i].id);
      live.erase(live.begin() + (std::ptrdiff_t)i);
    }
    CHECK(r.in_use() <= cap, "in_use %lld > cap", (long long)r.in_use());
    int64_t sum = 0;
    for (const Live &l : live) sum += l.bytes;
    CHECK(r.in_use() >= sum, "in_use %lld below live bytes %lld", (long long)r.in_use(), (long long)sum);
  }
  for (const Live &l : live) r.free(l.id);
  CHECK(r.in_use() == 0 && r.live_count() == 0, "ring not empty after freeing all");
}

int main(int argc, char **argv) {
  const uint64_t seed = argc > 1 ? strtoull(argv[1], nullptr, 10) : 1;
  std::mt19937_64 rng(seed);
  ring_check(rng);

  const int ks[3] = {7, 7, 9}, betas[3] = {2, 3, 2};
  std::vector<CodeShape> shapes;
  for (int c = 0; c < 3; ++c) {
    const int64_t L = 8 * (1 + (int64_t)(rng() % 64));
    const int64_t v = (int64_t)(rng() % 50);
    const int64_t v1 = (int64_t)(rng() % (uint64_t)(v + 1));
    shapes.push_back({ks[c], betas[c], L, v1, v - v1});
  }
  const int elem = rng() % 2 ? 1 : 4;
  const int64_t arena = 256 * (64 + (int64_t)(rng() % 4096));
  const int max_frames = 1 + (int)(rng() % 64);
  const int max_items = 1 + (int)(rng() % 300);
  Core core(shapes, arena, max_frames, max_items);

  struct Truth {
    Frame f;
    int64_t next_cs = 0;       // next core bit expected
    bool ingested = false, finished = false, admitted = false;
    int64_t admit_order = -1;
  };
  std::map<uint64_t, Truth> frames;
  std::deque<uint64_t> submit_order;
  int64_t admitted_so_far = 0;
  std::deque<Iteration> inflight;
  std::map<uint64_t, std::pair<int64_t, int64_t>> on_device;  // tag -> arena [off, end)
  uint64_t next_tag = 1;
  int64_t finished = 0, submitted = 0;
  const int64_t total = 300 + (int64_t)(rng() % 500);
  int64_t host_off = 0;

  for (int64_t step = 0; finished < total; ++step) {
    CHECK(step < 10000000, "no progress");
    if (step % 16 == 0) {  // the queue's block count: ceil(n / L) over the frames not yet admitted
      int64_t want = 0;
      for (const auto &kv : frames)
        if (!kv.second.admitted) want += (kv.second.f.n + shapes[kv.second.f.code].L - 1) / shapes[kv.second.f.code].L;
      CHECK(core.pending_blocks() == want, "pending blocks %lld, want %lld", (long long)core.pending_blocks(),
            (long long)want);
    }
    const int what = (int)(rng() % 4);
    if (what == 0 && submitted < total) {
      const int nsub = 1 + (int)(rng() % 8);
      for (int j = 0; j < nsub && submitted < total; ++j) {
        Frame f;
        f.tag = next_tag++;
        f.code = (int)(rng() % 3);
        f.terminated = (int)(rng() % 2);
        f.n = 1 + (int64_t)(rng() % 3000);
        f.N = f.n + (f.terminated ? ks[f.code] - 1 : 0);
        f.llr_bytes = f.N * betas[f.code] * elem;
        f.llr_src = host_off;
        f.out_dst = host_off + f.llr_bytes;
        host_off += f.llr_bytes + (f.n + 7) / 8;
        f.arrival_ns = step;
        if (!core.fits_ever(f)) continue;  // the server refuses these at submit
        core.submit(f);
        frames[f.tag].f = f;
        submit_order.push_back(f.tag);
        ++submitted;
      }
    } else if ((what == 1 || what == 0) && inflight.size() < 2) {
      Iteration it;
      VectorSink sink;
      if (!core.next_iteration(&it, sink)) {
        CHECK(sink.items.empty() && it.ingest.empty(), "empty iteration with work");
        continue;
      }
      const std::vector<Item> &items = sink.items;
      CHECK((int64_t)items.size() == it.nitems, "sink got %zu items, iteration says %lld", items.size(),
            (long long)it.nitems);
      for (int c = 0; c < 3; ++c)
        CHECK(std::count_if(items.begin(), items.end(), [&](const Item &b) { return b.code == c; }) == it.count[c],
              "per-code count");
      CHECK((int64_t)items.size() <= max_items, "%zu items > %d", items.size(), max_items);
      // ingest: admissions in FIFO order
      for (const Copy &c : it.ingest) {
        CHECK(!submit_order.empty(), "ingest with nothing submitted");
        const uint64_t tag = submit_order.front();
        submit_order.pop_front();
        Truth &t = frames[tag];
        CHECK(c.src == t.f.llr_src && c.bytes == t.f.llr_bytes, "ingest of frame %llu not in FIFO order",
              (unsigned long long)tag);
        CHECK(c.dst % 256 == 0 && c.dst >= 0, "ingest destination misaligned");
        const int64_t end = c.dst + ((c.bytes + 255) / 256) * 256;
        CHECK(end <= arena, "frame arena range beyond the arena");
        for (const auto &kv : on_device)
          CHECK(end <= kv.second.first || kv.second.second <= c.dst, "arena ranges of frames %llu and %llu overlap",
                (unsigned long long)tag, (unsigned long long)kv.first);
        on_device[tag] = {c.dst, end};
        t.ingested = true;
        t.admitted = true;
        t.admit_order = admitted_so_far++;
        t.f.arena_llr = c.dst;
      }
      CHECK((int64_t)on_device.size() <= max_frames, "%zu frames on device > %d", on_device.size(), max_frames);
      // items: geometry, order, grouping
      std::map<int64_t, uint64_t> by_arena;
      for (const auto &kv : on_device) by_arena[kv.second.first] = kv.first;
      for (size_t i = 0; i < items.size(); ++i) {
        const Item &b = items[i];
        if (i) {
          const Item &a = items[i - 1];
          CHECK(a.code <= b.code, "items not grouped by code");
        }
        CHECK(by_arena.count(b.llr_off), "item of a frame not on the device");
        Truth &t = frames[by_arena[b.llr_off]];
        CHECK(t.ingested && b.code == t.f.code && b.out_off == t.f.out_dst, "item addresses");
      }
      // per frame, blocks in order (items are sorted, so collect first)
      std::map<uint64_t, std::vector<Item>> per;
      for (const Item &b : items) per[by_arena[b.llr_off]].push_back(b);
      // fair share: when the iteration has room for one block per active
      // frame, every admitted frame with blocks left gets at least one
      int64_t waiting = 0;
      for (const auto &kv : frames)
        if (kv.second.admitted && kv.second.next_cs < kv.second.f.n) ++waiting;
      if (waiting <= max_items)
        for (const auto &kv : frames)
          if (kv.second.admitted && kv.second.next_cs < kv.second.f.n)
            CHECK(per.count(kv.first), "frame %llu got no block in an iteration with room for all",
                  (unsigned long long)kv.first);
      for (auto &kv : per) {
        Truth &t = frames[kv.first];
        const CodeShape &sh = shapes[t.f.code];
        std::sort(kv.second.begin(), kv.second.end(), [](const Item &a, const Item &b) { return a.cs < b.cs; });
        for (const Item &b : kv.second) {
          const int64_t cs = t.next_cs, ce = std::min(cs + sh.L, t.f.n);
          const int64_t s = std::max<int64_t>(0, cs - sh.v1), e = std::min(t.f.N, ce + sh.v2);
          CHECK(b.cs == cs && b.ce == ce && b.s == s && b.e == e && b.cost == e - s,
                "frame %llu block geometry: got cs %d ce %d s %d e %d, want %lld %lld %lld %lld",
                (unsigned long long)kv.first, b.cs, b.ce, b.s, b.e, (long long)cs, (long long)ce, (long long)s,
                (long long)e);
          CHECK(b.flags == ((s == 0 ? 1 : 0) | ((t.f.terminated && e == t.f.N) ? 2 : 0)), "flags");
          t.next_cs = ce;
        }
      }
      // finishing: exactly the frames whose last block is in this iteration
      std::set<uint64_t> fin;
      for (const Frame &f : it.finishing) fin.insert(f.tag);
      CHECK(fin.size() == it.finishing.size(), "a frame finishing twice in one iteration");
      for (size_t i = 0; i < it.finishing.size(); ++i) {
        Truth &t = frames[it.finishing[i].tag];
        CHECK(t.next_cs == t.f.n, "frame %llu finishing with bits left", (unsigned long long)t.f.tag);
        CHECK(per.count(t.f.tag), "frame %llu finishing without a block in the iteration", (unsigned long long)t.f.tag);
      }
      for (auto &kv : frames)
        if (kv.second.admitted && !kv.second.finished && kv.second.next_cs == kv.second.f.n)
          CHECK(fin.count(kv.first) || std::any_of(inflight.begin(), inflight.end(), [&](const Iteration &x) {
                  for (const Frame &f : x.finishing) if (f.tag == kv.first) return true;
                  return false;
                }), "frame %llu fully launched but never finishing", (unsigned long long)kv.first);
      inflight.push_back(it);
    } else if (!inflight.empty()) {
      Iteration &it = inflight.front();
      for (const Frame &f : it.finishing) {
        Truth &t = frames[f.tag];
        CHECK(!t.finished, "frame finished twice");
        t.finished = true;
        on_device.erase(f.tag);
        ++finished;
      }
      core.retire(it);
      inflight.pop_front();
      CHECK(core.frames_on_device() == (int64_t)on_device.size(), "frames on device %lld vs %zu",
            (long long)core.frames_on_device(), on_device.size());
    }
  }
  CHECK(!core.has_work() && inflight.empty() && core.arena_in_use() == 0 && core.pending_blocks() == 0,
        "work left at the end");

  // queue timeouts: expire_queued drops expired frames from the front of the
  // queue only (an early arrival behind a live frame waits for its turn)
  {
    Core q(shapes, arena, max_frames, max_items);
    const int64_t arrivals[5] = {5, 7, 20, 3, 30};
    for (int j = 0; j < 5; ++j) {
      Frame f;
      f.tag = 1000 + (uint64_t)j;
      f.code = 0;
      f.terminated = 1;
      f.n = 16;
      f.N = 22;
      f.llr_bytes = 44 * elem;
      f.llr_src = 0;
      f.out_dst = 0;
      f.arrival_ns = arrivals[j];
      CHECK(q.fits_ever(f), "timeout frame does not fit");
      q.submit(f);
    }
    std::vector<uint64_t> gone;
    auto note = [&](const Frame &f) { gone.push_back(f.tag); };
    CHECK(q.expire_queued(10, note) == 2 && gone.size() == 2 && gone[0] == 1000 && gone[1] == 1001,
          "expire at 10");
    const int64_t b16 = (16 + shapes[0].L - 1) / shapes[0].L;
    CHECK(q.pending() == 3 && q.pending_blocks() == 3 * b16, "pending after the first expiry");
    CHECK(q.expire_queued(25, note) == 2 && gone[2] == 1002 && gone[3] == 1003, "expire at 25");
    CHECK(q.pending() == 1 && q.expire_queued(30, note) == 0, "arrival 30 is not before 30");
    Iteration it;
    VectorSink sink;
    CHECK(q.next_iteration(&it, sink) && it.admitted == 1, "the remaining frame is admitted");
    CHECK(q.expire_queued(1000, note) == 0, "admitted frames never expire");
    q.retire(it);
    for (int rounds = 0; q.has_work() && rounds < 100; ++rounds) {  // blocks left for later iterations
      Iteration more;
      q.next_iteration(&more, sink);
      q.retire(more);
    }
    CHECK(!q.has_work() && q.arena_in_use() == 0, "timeout core left work");
  }

  // fail_all drops queued and admitted frames and frees their arena
  for (int j = 0; j < 20; ++j) {
    Frame f;
    f.tag = next_tag++;
    f.code = 0;
    f.terminated = 1;
    f.n = 100;
    f.N = 106;
    f.llr_bytes = 212 * elem;
    f.llr_src = 0;
    f.out_dst = 0;
    f.arrival_ns = 0;
    if (core.fits_ever(f)) core.submit(f);
  }
  Iteration it;
  VectorSink sink;
  core.next_iteration(&it, sink);
  int64_t dropped = 0;
  core.fail_all([&](const Frame &, bool) { ++dropped; });
  core.retire(it);
  CHECK(!core.has_work() && core.frames_on_device() == 0 && core.arena_in_use() == 0 && core.pending_blocks() == 0,
        "fail_all left work");
  // an exception at the checkpoint after admission: the admitted frames stay
  // counted (admitted_total, frames_on_device) and fail_all reports each of
  // them once, as admitted, and each queued one once, as queued
  {
    Core x(shapes, arena, max_frames, max_items);
    struct Boom {};
    static bool armed;
    armed = true;
    x.checkpoint = [] {
      if (armed) {
        armed = false;
        throw Boom();
      }
    };
    int64_t sent = 0;
    for (int j = 0; j < 3 * max_frames; ++j) {
      Frame f;
      f.tag = 5000 + (uint64_t)j;
      f.code = j % (int)shapes.size();
      f.terminated = 1;
      f.n = 24;
      f.N = f.n + shapes[f.code].k - 1;
      f.llr_bytes = f.N * shapes[f.code].beta * elem;
      f.llr_src = 0;
      f.out_dst = 0;
      f.arrival_ns = 0;
      if (!x.fits_ever(f)) continue;
      x.submit(f);
      ++sent;
    }
    Iteration it;
    VectorSink sink;
    bool threw = false;
    try {
      x.next_iteration(&it, sink);
    } catch (const Boom &) {
      threw = true;
    }
    CHECK(threw && x.admitted_total() > 0 && x.admitted_total() == x.frames_on_device(),
          "admissions before the exception: %lld counted, %lld on device", (long long)x.admitted_total(),
          (long long)x.frames_on_device());
    int64_t adm = 0, queued = 0;
    std::set<uint64_t> seen;
    x.fail_all([&](const Frame &f, bool a) {
      CHECK(seen.insert(f.tag).second, "frame %llu reported twice", (unsigned long long)f.tag);
      (a ? adm : queued) += 1;
    });
    CHECK(adm == x.admitted_total() && adm + queued == sent, "fail_all: %lld admitted + %lld queued of %lld",
          (long long)adm, (long long)queued, (long long)sent);
    CHECK(!x.has_work() && x.frames_on_device() == 0 && x.arena_in_use() == 0, "work left after the exception");
  }
  printf("OK seed %llu: %lld frames, arena %lld, slots %d, items/iter %d, L %lld/%lld/%lld\n",
         (unsigned long long)seed, (long long)finished, (long long)arena, max_frames, max_items,
         (long long)shapes[0].L, (long long)shapes[1].L, (long long)shapes[2].L);
  return 0;
}
