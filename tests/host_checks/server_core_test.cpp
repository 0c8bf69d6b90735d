// The continuous-batching server's policy (serve::Core) driven by a fake
// executor and a virtual clock: admission order under the HBM budget, LRU
// eviction that skips fields a request still names, merging of slider
// requests into one launch per free slot, sliders waiting for their field's
// upload, isolation of failed uploads and launches, and memory and latency
// bookkeeping.  Built with the host compiler only; exits non-zero on the
// first failed check.
#include <cstdio>
#include <cstdlib>
#include <map>
#include <memory>
#include <set>
#include <string>
#include <vector>

#include "../../paper_2510_01190_amd/csrc/server_core.hpp"

using namespace pdiv::serve;

static int g_checks = 0;
#define CHECK(c)                                                             \
  do {                                                                       \
    ++g_checks;                                                              \
    if (!(c)) {                                                              \
      std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
      std::exit(1);                                                          \
    }                                                                        \
  } while (0)

struct VirtualClock {
  double t = 0;
};

// Work finishes `duration` seconds of virtual time after it starts; an
// outcome of -1 makes poll report failure.  Start failures are scheduled by
// call number.
struct FakeExecutor : Executor {
  struct Job {
    double done_at;
    int outcome;
    bool upload;
    std::vector<uint64_t> tickets;
    int slot;
  };
  VirtualClock* clk;
  double upload_s = 0.010, slider_s = 0.002;
  std::map<uint64_t, Job> jobs;
  uint64_t next = 1;
  std::set<int> fail_upload_start, fail_upload_run, fail_slider_start, fail_slider_run;
  int uploads = 0, sliders = 0;
  std::vector<std::vector<uint64_t>> launches;  // tickets of each slider launch
  std::vector<int> launch_slots;
  std::vector<uint64_t> freed;                  // evicted field ids, in order
  std::set<void*> hosts_out;                    // host staging lent to the core
  std::set<int> busy_slots;
  int released = 0;

  explicit FakeExecutor(VirtualClock* c) : clk(c) {}

  uint64_t start_upload(Request* r, Field* f, size_t) override {
    ++uploads;
    CHECK(hosts_out.count(r->host) == 1);
    if (fail_upload_start.count(uploads)) return 0;
    f->dev[0] = f->dev[1] = reinterpret_cast<void*>(uintptr_t(0x1000 + f->id));
    jobs[next] = Job{clk->t + upload_s, fail_upload_run.count(uploads) ? -1 : 1, true,
                     {r->ticket}, -1};
    return next++;
  }
  uint64_t start_sliders(const std::vector<Request*>& reqs, const std::vector<Field*>& fs,
                         int slot) override {
    ++sliders;
    CHECK(reqs.size() == fs.size());
    CHECK(!reqs.empty() && int(reqs.size()) <= kMaxBatch);
    CHECK(busy_slots.count(slot) == 0);  // a slot is never used twice at once
    std::vector<uint64_t> t;
    for (size_t i = 0; i < reqs.size(); ++i) {
      CHECK(fs[i]->ready && !fs[i]->failed);
      CHECK(fs[i]->id == reqs[i]->fid);
      CHECK(fs[i]->dev[0] != nullptr);
      t.push_back(reqs[i]->ticket);
    }
    if (fail_slider_start.count(sliders)) return 0;
    launches.push_back(t);
    launch_slots.push_back(slot);
    busy_slots.insert(slot);
    jobs[next] = Job{clk->t + slider_s, fail_slider_run.count(sliders) ? -1 : 1, false, t, slot};
    return next++;
  }
  int poll(uint64_t h) override {
    const Job& j = jobs.at(h);
    if (clk->t < j.done_at) return 0;
    return j.outcome;
  }
  void release(uint64_t h) override {
    const Job& j = jobs.at(h);
    if (j.slot >= 0) busy_slots.erase(j.slot);
    jobs.erase(h);
    ++released;
  }
  void free_field(Field* f) override {
    freed.push_back(f->id);
    f->dev[0] = f->dev[1] = nullptr;
  }
  void return_host(void* host) override {
    CHECK(hosts_out.erase(host) == 1);  // each buffer comes back exactly once
  }
};

// A server around the core with the clock and request storage of a test.
struct Harness {
  static constexpr size_t kFixed = 1000;
  VirtualClock clk;
  FakeExecutor ex{&clk};
  Core core;
  std::vector<std::unique_ptr<Request>> reqs;
  std::vector<std::unique_ptr<char>> hosts;
  uint64_t ticket = 1;

  Harness(size_t budget, int n_slots)
      : core(budget, n_slots, kFixed, [this] { return clk.t; }) {}

  Request* put(uint64_t id, int ny, int nx, size_t dtype_bytes = 4) {
    auto r = std::make_unique<Request>();
    r->fid = id;
    r->ny = ny;
    r->nx = nx;
    r->dtype_bytes = dtype_bytes;
    r->t_submit = clk.t;
    r->ticket = ticket++;
    hosts.emplace_back(new char);
    r->host = hosts.back().get();
    ex.hosts_out.insert(r->host);
    CHECK(!core.has_field(id));
    core.add_new(r.get());
    reqs.push_back(std::move(r));
    return reqs.back().get();
  }
  Request* slide(uint64_t id, int n_iso = 4) {
    auto r = std::make_unique<Request>();
    r->fid = id;
    r->n_iso = n_iso;
    r->t_submit = clk.t;
    r->ticket = ticket++;
    if (!core.add_slider(r.get())) return nullptr;
    reqs.push_back(std::move(r));
    return reqs.back().get();
  }
  void step() { core.step(ex); }
  void advance(double s) {
    clk.t += s;
    step();
  }
  // Runs until nothing is queued or in flight (bounded).
  void drain() {
    for (int i = 0; i < 10000 && !core.idle(); ++i) advance(0.001);
    CHECK(core.idle());
  }
};

// field of ny x nx points: 8 bytes per point resident, 4 planes staged
static size_t res_bytes(int ny, int nx) { return 8 * size_t(ny) * size_t(nx); }
static size_t stg_bytes(int ny, int nx, size_t b = 4) { return 4 * b * size_t(ny) * size_t(nx); }

static void test_upload_then_sliders_merge() {
  Harness h(1 << 24, 2);
  Request* n1 = h.put(1, 64, 64);
  Request* s1 = h.slide(1);
  Request* s2 = h.slide(1, 16);
  CHECK(h.slide(99) == nullptr);  // not resident
  h.step();
  CHECK(h.ex.uploads == 1);
  CHECK(h.ex.sliders == 0);  // the field is still uploading
  CHECK(h.core.resident() == Harness::kFixed + res_bytes(64, 64) + stg_bytes(64, 64));
  h.advance(0.005);
  CHECK(!n1->done && h.ex.sliders == 0);
  h.advance(0.005);  // upload done at 10 ms: both sliders go in one launch
  CHECK(n1->done && n1->status == kOk);
  CHECK(h.core.resident() == Harness::kFixed + res_bytes(64, 64));  // staging returned
  CHECK(h.ex.hosts_out.empty());
  CHECK(h.ex.launches.size() == 1);
  CHECK((h.ex.launches[0] == std::vector<uint64_t>{s1->ticket, s2->ticket}));
  h.advance(0.002);
  CHECK(s1->done && s2->done && s1->status == kOk && s2->status == kOk);
  const Core::Stats st = h.core.stats();
  CHECK(st.done == 3 && st.failed == 0 && st.launches == 1);
  CHECK(st.cells == 63.0 * 63.0 * (4 + 16));
  CHECK(st.peak == Harness::kFixed + res_bytes(64, 64) + stg_bytes(64, 64));
  // latencies on the virtual clock: upload 10 ms, sliders 12 ms after submit
  CHECK(std::abs(st.p50_new_us - 10000.0) < 1e-6);
  CHECK(std::abs(st.p50_slider_us - 12000.0) < 1e-6);
  // all three: 10, 12, 12 ms -> median 12 ms, p99 interpolated to 12 ms
  CHECK(std::abs(st.p50_us - 12000.0) < 1e-6);
  CHECK(std::abs(st.p99_us - 12000.0) < 1e-6);
  CHECK(std::abs(st.p99_new_us - 10000.0) < 1e-6);
  std::printf("PASS upload_then_sliders_merge\n");
}

static void test_one_launch_per_free_slot() {
  Harness h(1 << 24, 2);
  h.put(1, 32, 32);
  h.put(2, 32, 48);
  h.drain();
  // 600 requests over two fields, queued while nothing runs: the first
  // launch takes kMaxBatch in arrival order, the second slot the rest
  std::vector<Request*> rs;
  for (int i = 0; i < 600; ++i) rs.push_back(h.slide(1 + i % 2, 1 + i % 16));
  h.step();
  CHECK(h.ex.launches.size() == 2);
  CHECK(h.ex.launches[0].size() == size_t(kMaxBatch));
  CHECK(h.ex.launches[1].size() == size_t(600 - kMaxBatch));
  CHECK(h.ex.launch_slots[0] != h.ex.launch_slots[1]);
  for (int i = 0; i < kMaxBatch; ++i) CHECK(h.ex.launches[0][size_t(i)] == rs[size_t(i)]->ticket);
  // both slots busy: new arrivals wait, then all go in the next free slot
  Request* late1 = h.slide(2);
  Request* late2 = h.slide(1);
  h.step();
  CHECK(h.ex.launches.size() == 2);
  h.advance(0.002);  // both launches finish; the two late requests merge
  CHECK(h.ex.launches.size() == 3);
  CHECK((h.ex.launches[2] == std::vector<uint64_t>{late1->ticket, late2->ticket}));
  h.drain();
  for (Request* r : rs) CHECK(r->done && r->status == kOk);
  CHECK(h.core.stats().launches == 3);
  std::printf("PASS one_launch_per_free_slot\n");
}

static void test_lru_eviction_skips_referenced() {
  const int n = 100;  // 100 x 100 points: 80 KB resident, 160 KB staged (f32)
  const size_t budget = Harness::kFixed + 3 * res_bytes(n, n) + stg_bytes(n, n);
  Harness h(budget, 1);
  h.put(1, n, n);
  h.drain();
  h.put(2, n, n);
  h.drain();
  h.put(3, n, n);
  h.drain();
  CHECK(h.ex.freed.empty());
  // last use (a put or a launch): 1 put, 2 put, 3 put, then 1 launched
  h.slide(1);
  h.drain();
  Request* busy = h.slide(3);  // 3 launched and in flight: the one slot is busy
  h.step();
  CHECK(!busy->done);
  Request* hold = h.slide(2);  // queued behind the busy slot: names field 2
  Request* n4 = h.put(4, n, n);
  h.step();
  // field 4 needs one field's room; 2 and 3 are named by requests, so the
  // victim is 1 although 2 was used less recently
  CHECK((h.ex.freed == std::vector<uint64_t>{1}));
  CHECK(!h.core.has_field(1));
  h.drain();
  CHECK(n4->status == kOk && hold->status == kOk);
  // last uses now: 3 launched, 4 put, 2 launched -> 3 is the oldest
  CHECK(h.core.field(3)->last_use < h.core.field(4)->last_use);
  CHECK(h.core.field(4)->last_use < h.core.field(2)->last_use);
  h.put(5, n, n);
  h.drain();
  CHECK((h.ex.freed == std::vector<uint64_t>{1, 3}));
  CHECK(h.core.resident() <= budget);
  CHECK(h.core.stats().peak <= budget);
  std::printf("PASS lru_eviction_skips_referenced\n");
}

static void test_fifo_admission_blocks_later_fields() {
  const int n = 100;
  // a 2n x n field with its staging fits only once field 1 is gone; a 10 x 10
  // field would fit beside field 1
  const size_t budget = Harness::kFixed + res_bytes(2 * n, n) + stg_bytes(2 * n, n) +
                        res_bytes(10, 10) + stg_bytes(10, 10);
  Harness h(budget, 1);
  h.put(1, n, n);
  h.drain();
  Request* hold = h.slide(1);
  h.step();  // launched: field 1 is named until it finishes
  CHECK(!hold->done);
  Request* big = h.put(2, 2 * n, n);
  Request* small = h.put(3, 10, 10);
  h.step();
  CHECK(h.ex.uploads == 1);  // neither admitted: big heads the queue
  CHECK(!big->done && !small->done);
  h.advance(0.002);  // hold finishes: 1 is evicted, then big and small go up
  CHECK(hold->done && hold->status == kOk);
  CHECK(h.ex.uploads == 3);
  CHECK((h.ex.freed == std::vector<uint64_t>{1}));
  h.drain();
  CHECK(big->status == kOk && small->status == kOk);
  CHECK(h.core.stats().peak == budget);
  std::printf("PASS fifo_admission_blocks_later_fields\n");
}

static void test_failed_upload_isolated() {
  Harness h(1 << 24, 2);
  h.ex.fail_upload_run.insert(2);    // field 2's reduction fails on the device
  h.ex.fail_upload_start.insert(3);  // field 3 cannot even be enqueued
  Request* a = h.put(1, 16, 16);
  Request* b = h.put(2, 16, 16);
  Request* sb = h.slide(2);
  Request* sa = h.slide(1);
  h.step();  // field 3 arrives after the first pass
  Request* c = h.put(3, 16, 16);
  Request* sc = h.slide(3);
  h.drain();
  CHECK(a->status == kOk && sa->status == kOk);
  CHECK(b->status == kDevice && sb->status == kDevice);
  CHECK(c->status == kDevice && sc->status == kDevice);
  CHECK(h.core.field(2)->failed && h.core.field(3)->failed);
  CHECK(h.ex.hosts_out.empty());  // every staging buffer came back
  // failed fields hold no staging; only their resident reservation
  CHECK(h.core.resident() == Harness::kFixed + 3 * res_bytes(16, 16));
  const Core::Stats st = h.core.stats();
  CHECK(st.done == 2 && st.failed == 4 && st.launches == 1);
  // the one slider launch held only the good request
  CHECK((h.ex.launches.back() == std::vector<uint64_t>{sa->ticket}));
  std::printf("PASS failed_upload_isolated\n");
}

static void test_failed_launch_isolated() {
  Harness h(1 << 24, 1);
  h.put(1, 16, 16);
  h.drain();
  h.ex.fail_slider_start.insert(1);  // nothing enqueued
  h.ex.fail_slider_run.insert(2);    // enqueued, fails on the device
  Request* r1 = h.slide(1);
  h.step();
  CHECK(r1->done && r1->status == kDevice);
  CHECK(h.ex.busy_slots.empty());  // the slot was not taken
  Request* r2 = h.slide(1);
  h.step();
  Request* r3 = h.slide(1);  // waits for the slot
  h.drain();
  CHECK(r2->status == kDevice && r3->status == kOk);
  CHECK(h.core.launches_issued() == 3);
  const Core::Stats st = h.core.stats();
  CHECK(st.launches == 2 && st.failed == 2);
  CHECK(st.cells == 15.0 * 15.0 * 4);  // only the good launch counts
  // refs all released: the field is evictable
  CHECK(h.core.field(1)->refs == 0);
  std::printf("PASS failed_launch_isolated\n");
}

static void test_shutdown_fails_queued() {
  const int n = 100;
  const size_t budget = Harness::kFixed + res_bytes(n, n) + stg_bytes(n, n);
  Harness h(budget, 1);
  h.put(1, n, n);
  h.drain();
  Request* s = h.slide(1);
  h.step();                           // launched; field 1 is referenced
  Request* r = h.put(2, n, n);        // cannot fit while 1 is referenced ...
  Request* s2 = h.slide(1);           // ... and 1 stays referenced by this
  h.ex.slider_s = 1e9;                // launches from here on never finish
  h.step();
  CHECK(!r->done);
  h.clk.t += 0.002;
  h.step();  // s finishes; s2 launches (slot free) and keeps field 1 named
  CHECK(s->done && s->status == kOk);
  CHECK(!h.core.nothing_in_flight());
  CHECK(!r->done);
  h.core.fail_queued(kBusy);
  CHECK(r->done && r->status == kBusy);
  CHECK(!s2->done);
  std::printf("PASS shutdown_fails_queued\n");
}

static void test_dtype_staging_bytes() {
  Harness h(1 << 24, 1);
  h.put(1, 50, 40, 2);  // 16-bit planes stage half the bytes
  h.step();
  CHECK(h.core.resident() == Harness::kFixed + res_bytes(50, 40) + stg_bytes(50, 40, 2));
  h.drain();
  CHECK(h.core.resident() == Harness::kFixed + res_bytes(50, 40));
  std::printf("PASS dtype_staging_bytes\n");
}

// Random arrivals against a small budget: invariants after every pass.
static void test_random_soak() {
  uint64_t x = 0x9E3779B97F4A7C15ull;
  auto rnd = [&x](uint64_t m) {
    x ^= x << 13;
    x ^= x >> 7;
    x ^= x << 17;
    return x % m;
  };
  const size_t budget = Harness::kFixed + 6 * res_bytes(64, 64);
  Harness h(budget, 3);
  h.ex.fail_upload_run.insert(7);
  h.ex.fail_slider_run.insert(11);
  uint64_t next_id = 1;
  std::vector<uint64_t> live;
  std::vector<Request*> all;
  for (int it = 0; it < 3000; ++it) {
    const uint64_t k = rnd(10);
    if (k == 0 && next_id < 200) {
      const int ny = 16 + int(rnd(48)), nx = 16 + int(rnd(48));
      all.push_back(h.put(next_id, ny, nx, rnd(2) ? 4 : 2));
      live.push_back(next_id++);
    } else if (k < 6 && !live.empty()) {
      Request* r = h.slide(live[rnd(live.size())], 1 + int(rnd(16)));
      if (r) all.push_back(r);
    }
    h.advance(0.0005 * double(rnd(4)));
    CHECK(h.core.resident() <= budget);
    for (size_t i = 0; i < live.size();)  // drop ids the core evicted
      if (!h.core.has_field(live[i])) live.erase(live.begin() + int64_t(i));
      else ++i;
  }
  h.drain();
  size_t ok = 0;
  for (Request* r : all) {
    CHECK(r->done);
    ok += r->status == kOk;
  }
  const Core::Stats st = h.core.stats();
  CHECK(st.done + st.failed == all.size());
  CHECK(st.done == ok);
  CHECK(st.peak <= budget);
  CHECK(h.ex.hosts_out.empty());
  CHECK(h.ex.jobs.empty());
  CHECK(h.ex.busy_slots.empty());
  std::printf("PASS random_soak (%zu requests, %llu launches, %zu evictions)\n", all.size(),
              (unsigned long long)st.launches, h.ex.freed.size());
}

int main() {
  test_upload_then_sliders_merge();
  test_one_launch_per_free_slot();
  test_lru_eviction_skips_referenced();
  test_fifo_admission_blocks_later_fields();
  test_failed_upload_isolated();
  test_failed_launch_isolated();
  test_shutdown_fails_queued();
  test_dtype_staging_bytes();
  test_random_soak();
  std::printf("ALL PASS (%d checks)\n", g_checks);
  return 0;
}
