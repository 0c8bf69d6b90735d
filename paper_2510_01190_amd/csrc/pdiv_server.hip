// Continuous-batching LCP server over device-resident fields.
//
// Fields arrive as host moment planes (pdiv_server_put_field): they are copied
// into pinned staging, uploaded on an upload stream, reduced to their
// divergence Gaussians (Eq. 2-3, 8 bytes per point) and kept resident.
// Isovalue-slider requests (pdiv_server_submit_lcp) name a resident field and
// 1..16 isovalues.  One worker thread runs the loop
//   completions -> admission of new fields by HBM budget (evicting least
//   recently used fields no request names) -> all slider requests waiting on
//   ready fields merged into one batched launch per free slot
// so requests that arrive while others are on the GPU join the next launch as
// soon as a slot frees; launches overlap on n_streams compute streams.  Each
// request's maps come from the same tile code as pdiv_lcp on the same
// divergence Gaussians, so a result is bitwise the same alone or in the mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "batch_internal.hpp"
#include "server_core.hpp"

using Clock = std::chrono::steady_clock;
using namespace pdiv;

namespace {

constexpr int kMaxBatch = serve::kMaxBatch;
constexpr int kBandRows = 16;    // tile height of server launches
constexpr int kMaxStreams = 8;
// Pinned staging buffers come in power-of-two size classes from 1 MiB up and
// are reused; the pool grows until it holds kDefaultPinnedCap bytes (or, after
// pdiv_server_reserve_staging, what it held then), after which a new field
// waits for a buffer to come back.  Fresh pinned pages fault on first touch (a few GB/s),
// so a pool that keeps growing under load costs far more than the copies.
constexpr size_t kPinnedClassMin = size_t(1) << 20;
constexpr size_t kDefaultPinnedCap = size_t(2) << 30;
constexpr int kCopyThreads = 4;            // host copy into staging
constexpr size_t kParallelCopyMin = size_t(8) << 20;

size_t pinned_class(size_t bytes) {
  size_t c = kPinnedClassMin;
  while (c < bytes) c <<= 1;
  return c;
}

// Copies (or, with src == nullptr, zero-fills) n_parts spans of `part` bytes,
// dst + i*part <- src[i], on up to kCopyThreads threads: one thread reaches
// about a third of the host-to-device DMA rate.
void staged_copy(char* dst, const void* const* src, int n_parts, size_t part) {
  const size_t total = part * size_t(n_parts);
  const int nt = total >= kParallelCopyMin ? kCopyThreads : 1;
  auto job = [&](int t) {
    for (int i = 0; i < n_parts; ++i) {
      const size_t lo = part * size_t(t) / nt, hi = part * size_t(t + 1) / nt;
      char* d = dst + size_t(i) * part + lo;
      if (src) std::memcpy(d, static_cast<const char*>(src[i]) + lo, hi - lo);
      else std::memset(d, 0, hi - lo);
    }
  };
  std::vector<std::thread> th;
  for (int t = 1; t < nt; ++t) th.emplace_back(job, t);
  job(0);
  for (auto& x : th) x.join();
}

size_t dtype_bytes(pdiv_dtype d) { return d == PDIV_F32 ? 4 : 2; }

struct PinnedBuf {
  void* p = nullptr;
  size_t bytes = 0;
  bool busy = false;
};

struct Slot {  // descriptor table + isovalues of one slider launch
  BatchField* dev_fields = nullptr;
  float* dev_iso = nullptr;
  BatchField* host_fields = nullptr;  // pinned
  float* host_iso = nullptr;          // pinned
};

struct Pending {  // device side of one in-flight handle
  hipEvent_t ev = nullptr;
  void* staging = nullptr;  // device staging of a new field
};

// Forced failures for tests of the failure paths, read when a server is
// created: PDIV_FAULT=<point>:<n>[,<point>:<n>] makes the n-th start (n >= 1)
// of <point> fail on the host before anything is enqueued.  Points:
// server_launch (a merged slider launch), server_upload (a new field's
// upload).  0 when <point> is not named.
int fault_after(const char* point) {
  const char* f = std::getenv("PDIV_FAULT");
  if (!f) return 0;
  const size_t len = std::strlen(point);
  for (const char* p = f; *p;) {
    if (std::strncmp(p, point, len) == 0 && p[len] == ':') return std::atoi(p + len + 1);
    const char* c = std::strchr(p, ',');
    if (!c) break;
    p = c + 1;
  }
  return 0;
}

double seconds_now() {
  return std::chrono::duration<double>(Clock::now().time_since_epoch()).count();
}

static_assert(serve::kMaxIso == kIsoChunk, "slider requests carry one isovalue chunk");

}  // namespace

// The policy (admission, eviction, merging, accounting) lives in serve::Core;
// this object is its device executor, the pinned staging pool and the worker.
struct pdiv_server_s : serve::Executor {
  int n_streams = 1;
  int device = 0;
  // private stream-ordered pool for resident fields and upload staging; it
  // keeps up to the budget mapped after frees, so admitting a field does not
  // map fresh pages while the worker holds the lock
  hipMemPool_t pool = nullptr;
  hipStream_t upload = nullptr;
  std::vector<hipStream_t> streams;
  std::vector<Slot> slots;
  size_t slot_bytes = 0;

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  bool stop = false;
  std::thread worker;

  std::unique_ptr<serve::Core> core;
  std::unordered_map<uint64_t, std::unique_ptr<serve::Request>> tickets;
  std::unordered_map<uint64_t, Pending> pending;
  uint64_t next_handle = 1;
  std::vector<std::unique_ptr<PinnedBuf>> pinned;
  size_t pinned_total = 0, pinned_cap = kDefaultPinnedCap;
  uint64_t next_ticket = 1;
  int next_stream = 0;
  int slider_starts = 0;
  int fault_at = 0;         // PDIV_FAULT server_launch
  int upload_starts = 0;
  int fault_upload_at = 0;  // PDIV_FAULT server_upload

  // --- pinned host staging (reused, released at destroy) -------------------
  PinnedBuf* alloc_pinned(size_t cls) {
    auto b = std::make_unique<PinnedBuf>();
    if (hipHostMalloc(&b->p, cls, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    b->bytes = cls;
    pinned_total += cls;
    pinned.push_back(std::move(b));
    return pinned.back().get();
  }

  bool any_pinned_busy() const {
    for (auto& b : pinned)
      if (b->busy) return true;
    return false;
  }

  // Called with mu held through lk.  Takes the smallest free buffer that
  // fits; else allocates within the cap, first releasing free buffers that
  // are too small; else waits for an upload to hand one back.  With nothing
  // busy the pool may pass the cap once, for a field larger than the cap.
  PinnedBuf* get_pinned(size_t bytes, std::unique_lock<std::mutex>& lk) {
    const size_t cls = pinned_class(bytes);
    while (true) {
      PinnedBuf* best = nullptr;
      for (auto& b : pinned)
        if (!b->busy && b->bytes >= cls && (!best || b->bytes < best->bytes)) best = b.get();
      if (!best) {
        for (size_t i = 0; i < pinned.size() && pinned_total + cls > pinned_cap;) {
          if (!pinned[i]->busy) {
            (void)hipHostFree(pinned[i]->p);
            pinned_total -= pinned[i]->bytes;
            pinned.erase(pinned.begin() + i);
          } else {
            ++i;
          }
        }
        if (pinned_total + cls <= pinned_cap || !any_pinned_busy()) {
          best = alloc_pinned(cls);
          if (!best) return nullptr;
        }
      }
      if (best) {
        best->busy = true;
        return best;
      }
      if (stop) return nullptr;
      cv_done.wait_for(lk, std::chrono::milliseconds(1));
    }
  }

  // --- serve::Executor (called by the core with mu held) --------------------
  uint64_t record(hipError_t e, hipStream_t s, void* staging) {
    Pending P;
    P.staging = staging;
    e = e != hipSuccess ? e : hipEventCreateWithFlags(&P.ev, hipEventDisableTiming);
    e = e != hipSuccess ? e : hipEventRecord(P.ev, s);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      if (P.ev) (void)hipEventDestroy(P.ev);
      if (staging) (void)hipFreeAsync(staging, upload);
      return 0;
    }
    const uint64_t h = next_handle++;
    pending[h] = P;
    return h;
  }

  uint64_t start_upload(serve::Request* r, serve::Field* f, size_t staging_bytes) override {
    if (fault_upload_at > 0 && ++upload_starts == fault_upload_at)
      return 0;  // forced from the host: nothing is allocated or enqueued
    const size_t n = size_t(r->ny) * size_t(r->nx);
    void* staging = nullptr;
    hipError_t e = hipMallocFromPoolAsync(&f->dev[0], 4 * n, pool, upload);
    e = e != hipSuccess ? e : hipMallocFromPoolAsync(&f->dev[1], 4 * n, pool, upload);
    e = e != hipSuccess ? e : hipMallocFromPoolAsync(&staging, staging_bytes, pool, upload);
    e = e != hipSuccess ? e
                        : hipMemcpyAsync(staging, static_cast<PinnedBuf*>(r->host)->p,
                                         staging_bytes, hipMemcpyHostToDevice, upload);
    const size_t pb = r->dtype_bytes * n;
    char* s = static_cast<char*>(staging);
    if (e == hipSuccess)
      e = launch_divergence(s, s + pb, s + 2 * pb, s + 3 * pb, pdiv_dtype(r->dtype), r->ny,
                            r->nx, make_coef(r->dx, r->dy), static_cast<float*>(f->dev[0]),
                            static_cast<float*>(f->dev[1]), upload);
    if (e != hipSuccess && staging) {
      (void)hipGetLastError();
      (void)hipFreeAsync(staging, upload);
      staging = nullptr;
    }
    return record(e, upload, staging);
  }

  uint64_t start_sliders(const std::vector<serve::Request*>& take,
                         const std::vector<serve::Field*>& fs, int slot) override {
    Slot& S = slots[size_t(slot)];
    int kc = 1;
    std::vector<BatchField> fv(take.size());
    for (size_t i = 0; i < take.size(); ++i) {
      const serve::Request* r = take[i];
      const serve::Field* f = fs[i];
      BatchField& x = fv[i];
      x = BatchField{};
      x.p0 = f->dev[0];
      x.p1 = f->dev[1];
      x.p2 = x.p3 = nullptr;
      x.lcp = r->out;
      x.iso = S.dev_iso + i * kIsoChunk;
      x.ny = f->ny;
      x.nx = f->nx;
      x.n_iso = r->n_iso;
      x.pitch = f->nx - 1;
      x.plane = int64_t(f->ny - 1) * x.pitch;
      x.coef = make_coef(f->dx, f->dy);
      std::memcpy(S.host_iso + i * kIsoChunk, r->iso, sizeof(float) * kIsoChunk);
      kc = std::max(kc, iso_bucket(r->n_iso));
    }
    const bool paired = kc >= 8 && all_rows_on_lines(fv);
    const int64_t n_tiles = fill_tiles(fv, kBandRows, paired);
    std::memcpy(S.host_fields, fv.data(), sizeof(BatchField) * fv.size());
    hipStream_t s = streams[size_t(next_stream)];
    next_stream = (next_stream + 1) % n_streams;
    const void* kernel = batch_kernel_ptr(false, PDIV_F32, kc, paired);
    const int grid =
        int(std::max<int64_t>(1, std::min<int64_t>(resident_blocks(kernel), (n_tiles + 3) / 4)));
    if (fault_at > 0 && ++slider_starts == fault_at)
      return 0;  // forced from the host: nothing is enqueued
    hipError_t e = hipMemcpyAsync(S.dev_fields, S.host_fields, sizeof(BatchField) * fv.size(),
                                  hipMemcpyHostToDevice, s);
    e = e != hipSuccess ? e
                        : hipMemcpyAsync(S.dev_iso, S.host_iso,
                                         sizeof(float) * kIsoChunk * fv.size(),
                                         hipMemcpyHostToDevice, s);
    e = e != hipSuccess
            ? e
            : launch_batch(kernel, S.dev_fields, int(fv.size()), n_tiles, kBandRows, grid, s);
    return record(e, s, nullptr);
  }

  int poll(uint64_t h) override {
    const hipError_t q = hipEventQuery(pending[h].ev);
    if (q == hipErrorNotReady) return 0;
    return q == hipSuccess ? 1 : -1;
  }

  void release(uint64_t h) override {
    auto it = pending.find(h);
    if (it->second.staging) (void)hipFreeAsync(it->second.staging, upload);
    (void)hipEventDestroy(it->second.ev);
    pending.erase(it);
  }

  void free_field(serve::Field* f) override {
    for (void*& p : f->dev)
      if (p) {
        (void)hipFreeAsync(p, upload);
        p = nullptr;
      }
  }

  void return_host(void* host) override { static_cast<PinnedBuf*>(host)->busy = false; }

  void run() {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    while (true) {
      core->step(*this);
      cv_done.notify_all();
      if (stop && core->idle()) break;
      if (core->nothing_in_flight()) {
        if (stop) {
          // nothing in flight and nothing admissible: fail what is left
          core->fail_queued(serve::kBusy);
          continue;
        }
        cv_work.wait(lk);
      } else {
        lk.unlock();
        std::this_thread::sleep_for(std::chrono::microseconds(20));
        lk.lock();
      }
    }
    cv_done.notify_all();
  }
};

extern "C" {

pdiv_status pdiv_server_create(size_t hbm_budget, int32_t n_streams, pdiv_server* out) {
  g_last_error.clear();
  if (out == nullptr) return invalid("out is NULL");
  *out = nullptr;
  if (n_streams < 1 || n_streams > kMaxStreams)
    return invalid("n_streams must be in [1, %d]", kMaxStreams);
  const int n_slots = 2 * n_streams;
  const size_t slot_bytes = kMaxBatch * (sizeof(BatchField) + sizeof(float) * kIsoChunk);
  if (hbm_budget < size_t(n_slots) * slot_bytes + (size_t(1) << 20))
    return invalid("hbm_budget too small (need more than %zu bytes)",
                   size_t(n_slots) * slot_bytes + (size_t(1) << 20));
  auto srv = std::make_unique<pdiv_server_s>();
  srv->n_streams = n_streams;
  srv->fault_at = fault_after("server_launch");
  srv->fault_upload_at = fault_after("server_upload");
  hipError_t e = hipGetDevice(&srv->device);
  hipMemPoolProps props{};
  props.allocType = hipMemAllocationTypePinned;
  props.location.type = hipMemLocationTypeDevice;
  props.location.id = srv->device;
  e = e != hipSuccess ? e : hipMemPoolCreate(&srv->pool, &props);
  uint64_t keep = hbm_budget;
  e = e != hipSuccess ? e
                      : hipMemPoolSetAttribute(srv->pool, hipMemPoolAttrReleaseThreshold, &keep);
  e = e != hipSuccess ? e : hipStreamCreateWithFlags(&srv->upload, hipStreamNonBlocking);
  for (int i = 0; i < n_streams && e == hipSuccess; ++i) {
    hipStream_t s = nullptr;
    e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess) srv->streams.push_back(s);
  }
  srv->slots.resize(n_slots);
  for (auto& S : srv->slots) {
    if (e != hipSuccess) break;
    e = hipMalloc(reinterpret_cast<void**>(&S.dev_fields), sizeof(BatchField) * kMaxBatch);
    e = e != hipSuccess ? e
                        : hipMalloc(reinterpret_cast<void**>(&S.dev_iso),
                                    sizeof(float) * kIsoChunk * kMaxBatch);
    e = e != hipSuccess ? e
                        : hipHostMalloc(reinterpret_cast<void**>(&S.host_fields),
                                        sizeof(BatchField) * kMaxBatch, hipHostMallocDefault);
    e = e != hipSuccess ? e
                        : hipHostMalloc(reinterpret_cast<void**>(&S.host_iso),
                                        sizeof(float) * kIsoChunk * kMaxBatch,
                                        hipHostMallocDefault);
  }
  srv->slot_bytes = size_t(n_slots) * slot_bytes;
  srv->core = std::make_unique<serve::Core>(hbm_budget, n_slots, srv->slot_bytes, seconds_now);
  pdiv_server raw = srv.release();
  if (e != hipSuccess) {
    device_status(e, "server create");
    pdiv_server_destroy(raw);
    set_error("server create: %s", hipGetErrorString(e));
    return PDIV_ERR_DEVICE;
  }
  raw->worker = std::thread([raw] { raw->run(); });
  *out = raw;
  return PDIV_OK;
}

pdiv_status pdiv_server_put_field(pdiv_server srv, uint64_t id, const void* mean_u_host,
                                  const void* var_u_host, const void* mean_v_host,
                                  const void* var_v_host, pdiv_dtype dtype, int64_t ny,
                                  int64_t nx, double dx, double dy, uint64_t* ticket) {
  g_last_error.clear();
  if (!srv || !mean_u_host || !var_u_host || !mean_v_host || !var_v_host || !ticket)
    return invalid("NULL argument");
  if (dtype != PDIV_F32 && dtype != PDIV_F16 && dtype != PDIV_BF16)
    return invalid("unknown dtype %d", int(dtype));
  if (ny < 2 || nx < 2 || ny > (int64_t(1) << 21) || nx > (int64_t(1) << 29))
    return invalid("bad grid %lld x %lld", (long long)ny, (long long)nx);
  if (!(std::isfinite(dx) && dx > 0) || !(std::isfinite(dy) && dy > 0))
    return invalid("dx and dy must be finite and > 0");
  const size_t n = size_t(ny) * size_t(nx), pb = dtype_bytes(dtype) * n;
  if (8 * n + 4 * pb + srv->slot_bytes > srv->core->budget()) {
    set_error("field of %zu points can never fit the %zu-byte budget", n, srv->core->budget());
    return PDIV_ERR_BUSY;
  }
  auto r = std::make_unique<serve::Request>();
  // latency counts from the call: waiting for staging and the host copy are
  // part of serving a new field
  r->t_submit = seconds_now();
  r->fid = id;
  r->dtype = dtype;
  r->dtype_bytes = dtype_bytes(dtype);
  r->ny = int(ny);
  r->nx = int(nx);
  r->dx = dx;
  r->dy = dy;
  PinnedBuf* host = nullptr;
  {
    std::unique_lock<std::mutex> lk(srv->mu);
    if (srv->stop) return invalid("server is shutting down");
    if (srv->core->has_field(id))
      return invalid("field id %llu is in use", (unsigned long long)id);
    host = srv->get_pinned(4 * pb, lk);
    if (!host) {
      set_error("cannot allocate %zu bytes of pinned staging", 4 * pb);
      return PDIV_ERR_NOMEM;
    }
    if (srv->core->has_field(id)) {  // taken while this call waited for staging
      host->busy = false;
      return invalid("field id %llu is in use", (unsigned long long)id);
    }
    // registered now (not yet queued) so that the id stays taken during the copy
    srv->core->reserve_field(r.get());
  }
  const void* const planes[4] = {mean_u_host, var_u_host, mean_v_host, var_v_host};
  staged_copy(static_cast<char*>(host->p), planes, 4, pb);
  r->host = host;
  {
    std::lock_guard<std::mutex> g(srv->mu);
    r->ticket = srv->next_ticket++;
    *ticket = r->ticket;
    srv->core->add_new(r.get());
    srv->tickets[r->ticket] = std::move(r);
  }
  srv->cv_work.notify_one();
  return PDIV_OK;
}

pdiv_status pdiv_server_reserve_staging(pdiv_server srv, int64_t max_points, pdiv_dtype dtype,
                                        int32_t count) {
  g_last_error.clear();
  if (!srv) return invalid("server is NULL");
  if (dtype != PDIV_F32 && dtype != PDIV_F16 && dtype != PDIV_BF16)
    return invalid("unknown dtype %d", int(dtype));
  if (max_points < 4 || max_points > (int64_t(1) << 40) || count < 1 || count > 64)
    return invalid("max_points must be in [4, 2^40] and count in [1, 64]");
  const size_t cls = pinned_class(4 * dtype_bytes(dtype) * size_t(max_points));
  std::vector<PinnedBuf*> fresh;
  {
    std::lock_guard<std::mutex> g(srv->mu);
    if (srv->stop) return invalid("server is shutting down");
    int have = 0;
    for (auto& b : srv->pinned)
      if (!b->busy && b->bytes >= cls) ++have;
    for (int i = have; i < count; ++i) {
      PinnedBuf* b = srv->alloc_pinned(cls);
      if (!b) {
        set_error("cannot allocate %zu bytes of pinned staging", cls);
        return PDIV_ERR_NOMEM;
      }
      b->busy = true;  // held while its pages are touched below
      fresh.push_back(b);
    }
    srv->pinned_cap = srv->pinned_total;  // the pool is now sized by the caller
  }
  for (PinnedBuf* b : fresh) staged_copy(static_cast<char*>(b->p), nullptr, 1, b->bytes);
  {
    std::lock_guard<std::mutex> g(srv->mu);
    for (PinnedBuf* b : fresh) b->busy = false;
  }
  return PDIV_OK;
}

pdiv_status pdiv_server_submit_lcp(pdiv_server srv, uint64_t id, const float* isovalues_host,
                                   int32_t n_iso, float* out, uint64_t* ticket) {
  g_last_error.clear();
  if (!srv || !isovalues_host || !out || !ticket) return invalid("NULL argument");
  if (n_iso < 1 || n_iso > kIsoChunk) return invalid("n_iso must be in [1, %d]", kIsoChunk);
  auto r = std::make_unique<serve::Request>();
  r->fid = id;
  r->n_iso = n_iso;
  for (int q = 0; q < kIsoChunk; ++q) r->iso[q] = isovalues_host[q < n_iso ? q : n_iso - 1];
  r->out = out;
  r->t_submit = seconds_now();
  {
    std::lock_guard<std::mutex> g(srv->mu);
    if (srv->stop) return invalid("server is shutting down");
    if (!srv->core->add_slider(r.get()))
      return invalid("field id %llu is not resident", (unsigned long long)id);
    r->ticket = srv->next_ticket++;
    *ticket = r->ticket;
    srv->tickets[r->ticket] = std::move(r);
  }
  srv->cv_work.notify_one();
  return PDIV_OK;
}

pdiv_status pdiv_server_wait(pdiv_server srv, uint64_t ticket, int64_t timeout_us,
                             pdiv_status* result) {
  g_last_error.clear();
  if (!srv || !result) return invalid("NULL argument");
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->tickets.find(ticket);
  if (it == srv->tickets.end()) return invalid("unknown ticket %llu", (unsigned long long)ticket);
  serve::Request* r = it->second.get();
  if (timeout_us < 0) {
    srv->cv_done.wait(lk, [&] { return r->done; });
  } else if (!srv->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us),
                                    [&] { return r->done; })) {
    return PDIV_ERR_TIMEOUT;
  }
  *result = pdiv_status(r->status);
  srv->tickets.erase(it);
  return PDIV_OK;
}

pdiv_status pdiv_server_stats(pdiv_server srv, pdiv_server_stats_t* out) {
  g_last_error.clear();
  if (!srv || !out) return invalid("NULL argument");
  std::lock_guard<std::mutex> g(srv->mu);
  const serve::Core::Stats s = srv->core->stats();
  out->done = s.done;
  out->failed = s.failed;
  out->launches = s.launches;
  out->p50_us = s.p50_us;
  out->p99_us = s.p99_us;
  out->p50_new_us = s.p50_new_us;
  out->p99_new_us = s.p99_new_us;
  out->p50_slider_us = s.p50_slider_us;
  out->p99_slider_us = s.p99_slider_us;
  out->lcp_cells = s.cells;
  out->resident_bytes = s.resident;
  out->peak_bytes = s.peak;
  return PDIV_OK;
}

pdiv_status pdiv_server_destroy(pdiv_server srv) {
  g_last_error.clear();
  if (!srv) return invalid("server is NULL");
  {
    std::lock_guard<std::mutex> g(srv->mu);
    srv->stop = true;
  }
  srv->cv_work.notify_all();
  if (srv->worker.joinable()) srv->worker.join();
  if (srv->core) srv->core->free_all(*srv);
  if (srv->upload) (void)hipStreamSynchronize(srv->upload);
  for (auto& S : srv->slots) {
    if (S.dev_fields) (void)hipFree(S.dev_fields);
    if (S.dev_iso) (void)hipFree(S.dev_iso);
    if (S.host_fields) (void)hipHostFree(S.host_fields);
    if (S.host_iso) (void)hipHostFree(S.host_iso);
  }
  for (auto& b : srv->pinned) (void)hipHostFree(b->p);
  for (hipStream_t s : srv->streams) (void)hipStreamDestroy(s);
  if (srv->upload) (void)hipStreamDestroy(srv->upload);
  if (srv->pool) (void)hipMemPoolDestroy(srv->pool);
  delete srv;
  return PDIV_OK;
}

}  // extern "C"
