// The continuous-batching server's policy, apart from the device: which new
// fields to admit under the HBM budget (first come, first served, evicting
// least recently used fields that no waiting request names), which slider
// requests to merge into a launch (every request waiting on a ready field,
// up to kMaxBatch, one launch per free descriptor slot), and the bookkeeping
// of completions, failures, memory and latency.  Plain host C++ with no HIP
// types: the device side is an Executor, so the policy runs unchanged
// against a fake executor and a virtual clock in a CPU test.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <deque>
#include <functional>
#include <memory>
#include <unordered_map>
#include <vector>

namespace pdiv {
namespace serve {

constexpr int kMaxBatch = 512;  // slider requests per launch
constexpr int kMaxIso = 16;     // isovalues per slider request

// Request outcome codes (the C ABI's pdiv_status values).
enum Status : int { kOk = 0, kInvalid = 1, kNoMem = 3, kDevice = 4, kBusy = 5 };

struct Field {
  uint64_t id = 0;
  int ny = 0, nx = 0;
  double dx = 1, dy = 1;
  size_t bytes = 0;       // resident bytes (its divergence Gaussians)
  bool ready = false;     // uploaded and reduced
  bool failed = false;    // its upload or reduction failed
  uint64_t last_use = 0;  // LRU stamp
  int refs = 0;           // requests (queued or in flight) that name it
  void* dev[2] = {nullptr, nullptr};  // the executor's device buffers
};

enum class Kind { kNew, kSlider };

struct Request {
  uint64_t ticket = 0;
  Kind kind = Kind::kSlider;
  uint64_t fid = 0;
  // new field: host staging (the executor's), storage, grid, spacing
  void* host = nullptr;
  int dtype = 0;
  size_t dtype_bytes = 4;
  int ny = 0, nx = 0;
  double dx = 1, dy = 1;
  // slider: isovalues and the caller's output
  float iso[kMaxIso] = {};
  int n_iso = 0;
  float* out = nullptr;
  double t_submit = 0;  // seconds, on the core's clock
  int status = kOk;
  bool done = false;
};

// What the policy asks of the device.  start_* enqueue work and return a
// handle (nonzero) or 0 if nothing could be enqueued; poll reports 1 once a
// handle's work has finished, -1 if it failed, 0 while it runs; release is
// called once per finished handle.
class Executor {
 public:
  virtual ~Executor() = default;
  // Allocate the field's resident buffers (f->bytes) and staging_bytes of
  // device staging, copy r->host there, reduce it to divergence Gaussians.
  virtual uint64_t start_upload(Request* r, Field* f, size_t staging_bytes) = 0;
  // One launch over the slider requests reqs (fields[i] is reqs[i]'s field)
  // with descriptor slot `slot`.
  virtual uint64_t start_sliders(const std::vector<Request*>& reqs,
                                 const std::vector<Field*>& fields, int slot) = 0;
  virtual int poll(uint64_t handle) = 0;
  virtual void release(uint64_t handle) = 0;
  // The field's resident buffers are no longer needed (evicted).
  virtual void free_field(Field* f) = 0;
  // A new field's host staging can be reused.
  virtual void return_host(void* host) = 0;
};

class Core {
 public:
  Core(size_t budget, int n_slots, size_t fixed_bytes, std::function<double()> now)
      : budget_(budget), slot_busy_(size_t(n_slots), false), now_(std::move(now)) {
    account(int64_t(fixed_bytes));
  }

  // --- requests (the caller holds the lock the server keeps around this) ---
  bool has_field(uint64_t id) const { return fields_.count(id) != 0; }
  Field* field(uint64_t id) {
    auto it = fields_.find(id);
    return it == fields_.end() ? nullptr : it->second.get();
  }
  // Takes a new field's id (not ready until uploaded; its request, named by
  // the field's one reference, follows with add_new).
  void reserve_field(const Request* r) {
    auto f = std::make_unique<Field>();
    f->id = r->fid;
    f->ny = r->ny;
    f->nx = r->nx;
    f->dx = r->dx;
    f->dy = r->dy;
    f->refs = 1;
    f->last_use = ++clock_;
    fields_[r->fid] = std::move(f);
  }
  // Queues a new field's request, reserving its id first if need be.
  void add_new(Request* r) {
    if (!has_field(r->fid)) reserve_field(r);
    r->kind = Kind::kNew;
    queue_.push_back(r);
  }
  // Queues a slider request; false if its field is not resident.
  bool add_slider(Request* r) {
    Field* f = field(r->fid);
    if (!f) return false;
    f->refs++;
    r->kind = Kind::kSlider;
    queue_.push_back(r);
    return true;
  }
  bool idle() const { return queue_.empty() && inflight_.empty(); }
  bool nothing_in_flight() const { return inflight_.empty(); }
  // Fails every queued request (shutting down with nothing admissible).
  void fail_queued(int status) {
    for (Request* r : queue_) finish(r, status);
    queue_.clear();
  }

  // --- one worker pass ------------------------------------------------------
  void step(Executor& ex) {
    poll_completions(ex);
    admit_new(ex);
    launch_sliders(ex);
  }

  void poll_completions(Executor& ex) {
    for (size_t i = 0; i < inflight_.size();) {
      Launch& L = inflight_[i];
      const int q = ex.poll(L.handle);
      if (q == 0) {
        ++i;
        continue;
      }
      const int st = q > 0 ? kOk : kDevice;
      for (Request* r : L.reqs) {
        if (r->kind == Kind::kNew) {
          Field* f = field(r->fid);
          if (f) f->ready = (st == kOk);
        }
        finish(r, st);
      }
      if (st == kOk) cells_ += L.cells;
      if (L.slot >= 0) slot_busy_[size_t(L.slot)] = false;
      if (L.staging_bytes) account(-int64_t(L.staging_bytes));
      if (L.host) ex.return_host(L.host);
      ex.release(L.handle);
      inflight_.erase(inflight_.begin() + int64_t(i));
    }
  }

  // Admits queued new fields in arrival order while the budget allows,
  // evicting least recently used idle fields; the first that cannot be made
  // to fit stops admission (later fields wait behind it).
  void admit_new(Executor& ex) {
    for (auto it = queue_.begin(); it != queue_.end();) {
      Request* r = *it;
      if (r->kind != Kind::kNew) {
        ++it;
        continue;
      }
      const size_t n = size_t(r->ny) * size_t(r->nx);
      const size_t res = 8 * n, stg = 4 * r->dtype_bytes * n;
      if (resident_ + res + stg > budget_ && !evict_for(res + stg, ex)) break;
      Field* f = field(r->fid);
      it = queue_.erase(it);
      f->bytes = res;
      account(int64_t(res + stg));
      const uint64_t h = ex.start_upload(r, f, stg);
      if (h == 0) {
        account(-int64_t(stg));
        ex.return_host(r->host);
        finish(r, kDevice);
        continue;
      }
      Launch L;
      L.handle = h;
      L.staging_bytes = stg;
      L.host = r->host;
      L.reqs.push_back(r);
      inflight_.push_back(L);
    }
  }

  // Merges every slider request waiting on a ready field into one launch per
  // free slot (at most kMaxBatch each); requests on a field that failed to
  // arrive fail.
  void launch_sliders(Executor& ex) {
    while (true) {
      int slot = -1;
      for (size_t i = 0; i < slot_busy_.size(); ++i)
        if (!slot_busy_[i]) {
          slot = int(i);
          break;
        }
      if (slot < 0) return;
      std::vector<Request*> take;
      std::vector<Field*> fs;
      for (auto it = queue_.begin(); it != queue_.end() && int(take.size()) < kMaxBatch;) {
        Request* r = *it;
        if (r->kind == Kind::kSlider) {
          Field* f = field(r->fid);
          if (f && f->failed) {
            it = queue_.erase(it);
            finish(r, kDevice);
            continue;
          }
          if (f && f->ready) {
            take.push_back(r);
            fs.push_back(f);
            it = queue_.erase(it);
            continue;
          }
        }
        ++it;
      }
      if (take.empty()) return;
      double cells = 0;
      for (size_t i = 0; i < take.size(); ++i) {
        fs[i]->last_use = ++clock_;
        cells += double(fs[i]->ny - 1) * double(fs[i]->nx - 1) * take[i]->n_iso;
      }
      ++launches_issued_;
      const uint64_t h = ex.start_sliders(take, fs, slot);
      if (h == 0) {
        for (Request* r : take) finish(r, kDevice);
        continue;
      }
      ++launches_;
      slot_busy_[size_t(slot)] = true;
      Launch L;
      L.handle = h;
      L.slot = slot;
      L.reqs = take;
      L.cells = cells;
      inflight_.push_back(L);
    }
  }

  // Frees every resident field (shutdown).
  void free_all(Executor& ex) {
    for (auto& kv : fields_) ex.free_field(kv.second.get());
  }

  // --- statistics ----------------------------------------------------------
  struct Stats {
    uint64_t done, failed, launches;
    double p50_us, p99_us, p50_new_us, p99_new_us, p50_slider_us, p99_slider_us, cells;
    size_t resident, peak;
  };
  Stats stats() const {
    std::vector<double> all = lat_new_;
    all.insert(all.end(), lat_slider_.begin(), lat_slider_.end());
    return Stats{done_,
                 failed_,
                 launches_,
                 pct(all, 0.50),
                 pct(all, 0.99),
                 pct(lat_new_, 0.50),
                 pct(lat_new_, 0.99),
                 pct(lat_slider_, 0.50),
                 pct(lat_slider_, 0.99),
                 cells_,
                 resident_,
                 peak_};
  }
  size_t resident() const { return resident_; }
  size_t budget() const { return budget_; }
  int launches_issued() const { return launches_issued_; }
  double now() const { return now_(); }

 private:
  struct Launch {
    uint64_t handle = 0;
    std::vector<Request*> reqs;
    int slot = -1;
    size_t staging_bytes = 0;
    void* host = nullptr;
    double cells = 0;
  };

  void account(int64_t delta) {
    resident_ = size_t(int64_t(resident_) + delta);
    peak_ = std::max(peak_, resident_);
  }

  void finish(Request* r, int st) {
    r->status = st;
    r->done = true;
    const double us = (now_() - r->t_submit) * 1e6;
    if (st == kOk) {
      ++done_;
      (r->kind == Kind::kNew ? lat_new_ : lat_slider_).push_back(us);
    } else {
      ++failed_;
    }
    Field* f = field(r->fid);
    if (f) {
      f->refs--;
      if (r->kind == Kind::kNew && st != kOk) f->failed = true;
    }
  }

  bool evict_for(size_t need, Executor& ex) {
    while (resident_ + need > budget_) {
      Field* victim = nullptr;
      for (auto& kv : fields_) {
        Field* f = kv.second.get();
        if ((f->ready || f->failed) && f->refs == 0 &&
            (!victim || f->last_use < victim->last_use))
          victim = f;
      }
      if (!victim) return false;
      ex.free_field(victim);
      account(-int64_t(victim->bytes));
      fields_.erase(victim->id);
    }
    return true;
  }

  static double pct(std::vector<double> v, double p) {
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    const double r = p * double(v.size() - 1);
    const size_t a = size_t(std::floor(r)), b = std::min(v.size() - 1, a + 1);
    return v[a] + (v[b] - v[a]) * (r - double(a));
  }

  size_t budget_;
  size_t resident_ = 0, peak_ = 0;
  std::vector<bool> slot_busy_;
  std::function<double()> now_;
  std::unordered_map<uint64_t, std::unique_ptr<Field>> fields_;
  std::deque<Request*> queue_;
  std::vector<Launch> inflight_;
  uint64_t clock_ = 0;
  uint64_t done_ = 0, failed_ = 0, launches_ = 0;
  int launches_issued_ = 0;
  double cells_ = 0;
  std::vector<double> lat_new_, lat_slider_;
};

}  // namespace serve
}  // namespace pdiv
