// Request server of the C ABI (ch_serve_*): continuous batching of host-side
// point sets over several streams, each stream owning one slot of the
// caller's device arena. Host code only; the hulls are computed by
// ch_hull_batch (and ch_hull for a set the batch rounds could not finish).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/convhull.h"
#include "ch_internal.hpp"

using chk::align_up;

namespace chk {
int ctx_device(const ch_ctx* ctx);
}

namespace {

constexpr uint32_t kDefaultInflight = 65536;
constexpr int kDefaultStreams = 4;
constexpr int kMaxStreams = 16;
constexpr uint32_t kMaxBatchSets = 65536;
// Requests of at most this many bytes are packed into pinned staging and
// copied with one DMA per batch; larger ones are copied from the caller's
// buffer directly.
constexpr size_t kStageReq = 64 << 10;
constexpr size_t kStageBytes = 8 << 20;
constexpr size_t kPinHull = 1 << 20;  // hull indices fetched through pinned memory

uint64_t now_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct Request {
  const float* h_xy = nullptr;
  uint32_t n = 0;
  ch_status status = CH_OK;
  bool done = false;
  bool waiting = false;
  std::vector<uint32_t> hull;
  uint64_t t_arrive = 0, t_admit = 0, t_done = 0;
};

// Device bytes one batch of `sets` requests with `points` points in total
// needs in a slot, when the largest single request's ch_hull workspace is
// `fallback` bytes.
size_t batch_need(uint64_t sets, uint64_t points, size_t fallback) {
  const size_t ws = std::max(chk::batch_layout((uint32_t)sets, points).total, fallback);
  return align_up(8 * points, 256) + align_up(8 * (sets + 1), 256) + align_up(4 * points, 256) +
         align_up(4 * sets, 256) + ws;
}

size_t fallback_ws(uint32_t n) { return n ? chk::layout(n).total : 0; }

size_t slot_bytes_of(const ch_serve_config* cfg) {
  const int k = cfg->n_streams ? cfg->n_streams : kDefaultStreams;
  if (k < 1 || k > kMaxStreams) return 0;
  return cfg->arena_bytes / (size_t)k / 256 * 256;
}

uint64_t max_points_for_slot(size_t slot) {
  if (batch_need(1, 1, fallback_ws(1)) > slot) return 0;
  uint64_t lo = 1, hi = CH_MAX_POINTS;
  while (lo < hi) {  // largest n with batch_need(1, n) <= slot
    const uint64_t mid = lo + (hi - lo + 1) / 2;
    if (batch_need(1, mid, fallback_ws((uint32_t)mid)) <= slot) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

}  // namespace

struct ch_server;

namespace {

struct Slot {
  ch_server* srv = nullptr;
  ch_ctx* ctx = nullptr;
  hipStream_t stream = nullptr;
  unsigned char* d_base = nullptr;
  unsigned char* pin_stage = nullptr;  // kStageBytes
  uint64_t* pin_off = nullptr;         // kMaxBatchSets + 1
  uint32_t* pin_cnt = nullptr;         // kMaxBatchSets
  uint32_t* pin_hull = nullptr;        // kPinHull
  std::thread th;
};

}  // namespace

struct ch_server {
  int device = 0;
  size_t slot_bytes = 0;
  uint64_t max_req = 0;
  uint64_t max_batch_points = 0;
  uint32_t max_inflight = kDefaultInflight;
  std::vector<Slot> slots;

  std::mutex mu;
  std::condition_variable cv_work;  // queue or stop
  std::condition_variable cv_done;  // a request finished, a waiter left
  std::deque<Request*> queue;
  std::unordered_map<uint64_t, Request*> tickets;
  uint64_t next_ticket = 1;
  uint32_t inflight = 0;
  bool stopping = false;
  int active_waiters = 0;

  uint64_t completed = 0, batches = 0;
  uint64_t first_arrive = 0, last_done = 0;
  std::vector<uint64_t> lat_ns;
};

namespace {

// Takes the next batch from the queue (caller holds the lock): requests in
// arrival order while the batch still fits the slot and the point cap.
std::vector<Request*> take_batch(ch_server* s) {
  std::vector<Request*> b;
  uint64_t pts = 0;
  size_t fb = 0;
  while (!s->queue.empty() && b.size() < kMaxBatchSets) {
    Request* r = s->queue.front();
    const uint64_t p2 = pts + r->n;
    const size_t fb2 = std::max(fb, fallback_ws(r->n));
    if (!b.empty()) {
      if (batch_need(b.size() + 1, p2, fb2) > s->slot_bytes) break;
      if (s->max_batch_points && p2 > s->max_batch_points) break;
    }
    b.push_back(r);
    s->queue.pop_front();
    pts = p2;
    fb = fb2;
  }
  return b;
}

void finish(ch_server* s, const std::vector<Request*>& b) {
  const uint64_t t = now_ns();
  std::lock_guard<std::mutex> lk(s->mu);
  for (Request* r : b) {
    r->t_done = t;
    r->done = true;
    s->completed += 1;
    s->lat_ns.push_back(t - r->t_arrive);
    if (!s->first_arrive || r->t_arrive < s->first_arrive) s->first_arrive = r->t_arrive;
  }
  s->last_done = t;
  s->batches += 1;
  s->cv_done.notify_all();
}

void fail_all(std::vector<Request*>& b, ch_status st) {
  for (Request* r : b) {
    r->status = st;
    r->hull.clear();
  }
}

// Runs one batch on the slot's stream and fills every request's result.
void run_batch(Slot& sl, std::vector<Request*>& b) {
  ch_server* s = sl.srv;
  const uint64_t t_admit = now_ns();
  for (Request* r : b) r->t_admit = t_admit;
  // Small requests first (staged), then the rest, each set's offset in order.
  std::stable_partition(b.begin(), b.end(),
                        [](const Request* r) { return size_t(r->n) * 8 <= kStageReq; });
  const uint32_t nsets = (uint32_t)b.size();
  uint64_t total = 0;
  size_t fb = 0;
  for (uint32_t i = 0; i < nsets; ++i) {
    sl.pin_off[i] = total;
    total += b[i]->n;
    fb = std::max(fb, fallback_ws(b[i]->n));
  }
  sl.pin_off[nsets] = total;

  unsigned char* p = sl.d_base;
  float* d_xy = reinterpret_cast<float*>(p);             p += align_up(8 * total, 256);
  uint64_t* d_off = reinterpret_cast<uint64_t*>(p);      p += align_up(8 * (uint64_t(nsets) + 1), 256);
  uint32_t* d_hidx = reinterpret_cast<uint32_t*>(p);     p += align_up(4 * total, 256);
  uint32_t* d_cnt = reinterpret_cast<uint32_t*>(p);      p += align_up(4 * uint64_t(nsets), 256);
  void* d_ws = p;
  const size_t ws_bytes = std::max(chk::batch_layout(nsets, total).total, fb);

  hipStream_t st = sl.stream;
  hipError_t e = hipSuccess;
  // Staged copies: pack the small requests, then one DMA.
  size_t staged = 0;
  uint32_t i = 0;
  auto flush = [&](uint32_t first_set) {
    if (staged && e == hipSuccess) {
      e = hipMemcpyAsync(reinterpret_cast<unsigned char*>(d_xy) + 8 * sl.pin_off[first_set],
                         sl.pin_stage, staged, hipMemcpyHostToDevice, st);
      // The staging buffer is reused only after this copy has finished.
      if (e == hipSuccess) e = hipStreamSynchronize(st);
    }
    staged = 0;
  };
  uint32_t run_first = 0;
  for (; i < nsets && size_t(b[i]->n) * 8 <= kStageReq; ++i) {
    const size_t bytes = size_t(b[i]->n) * 8;
    if (staged + bytes > kStageBytes) {
      flush(run_first);
      run_first = i;
    }
    if (bytes) std::memcpy(sl.pin_stage + staged, b[i]->h_xy, bytes);
    staged += bytes;
  }
  flush(run_first);
  for (; i < nsets && e == hipSuccess; ++i)
    if (b[i]->n)
      e = hipMemcpyAsync(reinterpret_cast<unsigned char*>(d_xy) + 8 * sl.pin_off[i], b[i]->h_xy,
                         size_t(b[i]->n) * 8, hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_off, sl.pin_off, 8 * (size_t(nsets) + 1), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) {
    fail_all(b, CH_E_DEVICE);
    return;
  }
  if (ch_hull_batch(sl.ctx, d_xy, d_off, nsets, total, d_hidx, d_cnt, d_ws, ws_bytes, st) != CH_OK) {
    fail_all(b, CH_E_DEVICE);
    return;
  }
  e = hipMemcpyAsync(sl.pin_cnt, d_cnt, 4 * size_t(nsets), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    fail_all(b, CH_E_DEVICE);
    return;
  }
  // Hull indices: through pinned memory while it has room, else directly.
  size_t pin_used = 0;
  std::vector<std::pair<uint32_t, size_t>> via_pin;  // (set, pinned position)
  for (uint32_t k = 0; k < nsets; ++k) {
    Request* r = b[k];
    const uint32_t c = sl.pin_cnt[k];
    if (c == CH_COUNT_DOMAIN_ERROR) {
      r->status = CH_E_DOMAIN;
    } else if (c > r->n) {
      r->status = CH_E_DEVICE;
    } else {
      r->status = CH_OK;
      r->hull.resize(c);
      if (!c) continue;
      if (pin_used + c <= kPinHull) {
        e = hipMemcpyAsync(sl.pin_hull + pin_used, d_hidx + sl.pin_off[k], 4 * size_t(c),
                           hipMemcpyDeviceToHost, st);
        via_pin.push_back({k, pin_used});
        pin_used += c;
      } else {
        e = hipMemcpyAsync(r->hull.data(), d_hidx + sl.pin_off[k], 4 * size_t(c),
                           hipMemcpyDeviceToHost, st);
      }
      if (e != hipSuccess) break;
    }
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    fail_all(b, CH_E_DEVICE);
    return;
  }
  for (auto& v : via_pin)
    std::memcpy(b[v.first]->hull.data(), sl.pin_hull + v.second, 4 * b[v.first]->hull.size());
  (void)s;
}

void worker(Slot* sl) {
  ch_server* s = sl->srv;
  (void)hipSetDevice(s->device);
  for (;;) {
    std::vector<Request*> b;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_work.wait(lk, [&] { return s->stopping || !s->queue.empty(); });
      if (s->stopping) return;
      b = take_batch(s);
    }
    if (b.empty()) continue;
    run_batch(*sl, b);
    finish(s, b);
  }
}

void destroy_slots(ch_server* s) {
  for (Slot& sl : s->slots) {
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
    if (sl.ctx) ch_ctx_destroy(sl.ctx);
    if (sl.pin_stage) (void)hipHostFree(sl.pin_stage);
    if (sl.pin_off) (void)hipHostFree(sl.pin_off);
    if (sl.pin_cnt) (void)hipHostFree(sl.pin_cnt);
    if (sl.pin_hull) (void)hipHostFree(sl.pin_hull);
  }
  s->slots.clear();
}

}  // namespace

extern "C" {

uint64_t ch_serve_max_request_points(const ch_serve_config* cfg) {
  if (!cfg) return 0;
  const size_t slot = slot_bytes_of(cfg);
  if (!slot) return 0;
  uint64_t m = max_points_for_slot(slot);
  if (cfg->max_batch_points && m > cfg->max_batch_points) m = cfg->max_batch_points;
  return m;
}

ch_status ch_serve_start(ch_ctx* ctx, const ch_serve_config* cfg, ch_server** out) {
  if (!ctx || !cfg || !out) return CH_E_INVALID_ARG;
  *out = nullptr;
  const int k = cfg->n_streams ? cfg->n_streams : kDefaultStreams;
  if (k < 1 || k > kMaxStreams) return CH_E_INVALID_ARG;
  if (!cfg->d_arena || (reinterpret_cast<uintptr_t>(cfg->d_arena) & 255u)) return CH_E_INVALID_ARG;
  const size_t slot = slot_bytes_of(cfg);
  if (!slot || max_points_for_slot(slot) == 0) return CH_E_INVALID_ARG;
  const int dev = chk::ctx_device(ctx);
  ch_server* s = new (std::nothrow) ch_server();
  if (!s) return CH_E_NOMEM;
  s->device = dev;
  s->slot_bytes = slot;
  s->max_req = ch_serve_max_request_points(cfg);
  s->max_batch_points = cfg->max_batch_points;
  s->max_inflight = cfg->max_inflight ? cfg->max_inflight : kDefaultInflight;
  s->slots.resize(k);
  ch_status err = CH_OK;
  for (int i = 0; i < k && err == CH_OK; ++i) {
    Slot& sl = s->slots[i];
    sl.srv = s;
    sl.d_base = static_cast<unsigned char*>(cfg->d_arena) + size_t(i) * slot;
    if (ch_ctx_create(dev, nullptr, &sl.ctx) != CH_OK) { err = CH_E_DEVICE; break; }
    if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess) { err = CH_E_DEVICE; break; }
    if (hipHostMalloc(reinterpret_cast<void**>(&sl.pin_stage), kStageBytes, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&sl.pin_off), 8 * (size_t(kMaxBatchSets) + 1),
                      hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&sl.pin_cnt), 4 * size_t(kMaxBatchSets),
                      hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&sl.pin_hull), 4 * kPinHull, hipHostMallocDefault) != hipSuccess)
      err = CH_E_NOMEM;
  }
  if (err != CH_OK) {
    destroy_slots(s);
    delete s;
    return err;
  }
  for (Slot& sl : s->slots) sl.th = std::thread(worker, &sl);
  *out = s;
  return CH_OK;
}

ch_status ch_serve_submit(ch_server* s, const float* h_xy, uint32_t n, uint64_t* ticket) {
  if (!s || !ticket || (n && !h_xy)) return CH_E_INVALID_ARG;
  if (n > s->max_req) return CH_E_INVALID_ARG;
  Request* r = new (std::nothrow) Request();
  if (!r) return CH_E_NOMEM;
  r->h_xy = h_xy;
  r->n = n;
  r->t_arrive = now_ns();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stopping) {
      delete r;
      return CH_E_SHUTDOWN;
    }
    if (s->inflight >= s->max_inflight) {
      delete r;
      return CH_E_BUSY;
    }
    const uint64_t t = s->next_ticket++;
    s->tickets.emplace(t, r);
    s->queue.push_back(r);
    s->inflight += 1;
    *ticket = t;
  }
  s->cv_work.notify_one();
  return CH_OK;
}

ch_status ch_serve_wait(ch_server* s, uint64_t ticket, int64_t timeout_us, uint32_t* hull_idx,
                        uint32_t cap, uint32_t* h_out, uint64_t* t_ns) {
  if (!s || !h_out || (cap && !hull_idx)) return CH_E_INVALID_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return CH_E_NOT_FOUND;
  Request* r = it->second;
  if (r->waiting) return CH_E_INVALID_ARG;
  r->waiting = true;
  s->active_waiters += 1;
  auto leave = [&](ch_status st) {
    s->active_waiters -= 1;
    s->cv_done.notify_all();
    return st;
  };
  if (timeout_us < 0) {
    s->cv_done.wait(lk, [&] { return r->done; });
  } else {
    s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), [&] { return r->done; });
  }
  if (!r->done) {
    r->waiting = false;
    return leave(CH_E_TIMEOUT);
  }
  if (r->status == CH_OK) {
    const uint32_t h = (uint32_t)r->hull.size();
    *h_out = h;
    if (h > cap) {
      r->waiting = false;
      return leave(CH_E_CAPACITY);
    }
    if (h) std::memcpy(hull_idx, r->hull.data(), 4 * size_t(h));
  }
  if (t_ns) {
    t_ns[0] = r->t_arrive;
    t_ns[1] = r->t_admit;
    t_ns[2] = r->t_done;
  }
  const ch_status st = r->status;
  s->tickets.erase(it);
  s->inflight -= 1;
  delete r;
  return leave(st);
}

ch_status ch_serve_stats(ch_server* s, uint64_t* completed, uint64_t* batches, double* hulls_per_s,
                         double* p50_us, double* p99_us) {
  if (!s) return CH_E_INVALID_ARG;
  std::vector<uint64_t> lat;
  uint64_t c, nb, t0, t1;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    lat = s->lat_ns;
    c = s->completed;
    nb = s->batches;
    t0 = s->first_arrive;
    t1 = s->last_done;
  }
  if (completed) *completed = c;
  if (batches) *batches = nb;
  if (hulls_per_s) *hulls_per_s = (c && t1 > t0) ? double(c) / (double(t1 - t0) * 1e-9) : 0.0;
  // Nearest-rank percentiles.
  auto pct = [&](double q) -> double {
    if (lat.empty()) return 0.0;
    size_t rank = (size_t)std::ceil(q / 100.0 * double(lat.size()));
    if (rank < 1) rank = 1;
    std::nth_element(lat.begin(), lat.begin() + (rank - 1), lat.end());
    return double(lat[rank - 1]) * 1e-3;
  };
  if (p50_us) *p50_us = pct(50.0);
  if (p99_us) *p99_us = pct(99.0);
  return CH_OK;
}

ch_status ch_serve_stop(ch_server* s) {
  if (!s) return CH_E_INVALID_ARG;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stopping = true;
    const uint64_t t = now_ns();
    for (Request* r : s->queue) {
      r->status = CH_E_SHUTDOWN;
      r->t_done = t;
      r->done = true;
    }
    s->queue.clear();
  }
  s->cv_work.notify_all();
  for (Slot& sl : s->slots)
    if (sl.th.joinable()) sl.th.join();
  {
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.notify_all();
    s->cv_done.wait(lk, [&] { return s->active_waiters == 0; });
    for (auto& kv : s->tickets) delete kv.second;
    s->tickets.clear();
  }
  destroy_slots(s);
  delete s;
  return CH_OK;
}

}  // extern "C"
