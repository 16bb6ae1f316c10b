// Request server of the C ABI (ch_serve_*): continuous batching of host-side
// point sets over several streams, each stream owning one slot of the
// caller's device arena. Host code only: the queue, tickets, batching and
// statistics are the Scheduler of ch_sched.hpp; each worker moves its batch
// to the device, runs ch_hull_batch and fetches the hulls.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <new>
#include <thread>
#include <vector>

#include "../../include/convhull.h"
#include "ch_internal.hpp"
#include "ch_sched.hpp"

using chk::align_up;
using chs::Request;

namespace chk {
int ctx_device(const ch_ctx* ctx);
}

namespace {

constexpr uint32_t kDefaultInflight = 65536;
constexpr int kDefaultStreams = 4;
constexpr int kMaxStreams = 16;
constexpr uint32_t kMaxBatchSets = 65536;
// Requests of at most this many bytes are packed into pinned staging and
// copied with one DMA per staging buffer; larger ones are copied from the
// caller's buffer directly. Two staging buffers alternate, so packing one
// overlaps the copy of the other.
constexpr size_t kStageReq = 64 << 10;
constexpr size_t kStageBytes = 8 << 20;
constexpr size_t kPinHull = 1 << 20;  // hull indices fetched through pinned memory

uint64_t now_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// Device bytes one batch of `sets` requests with `points` points in total
// needs in a slot: points, offsets, hull indices, counts and the batch
// workspace.
size_t batch_need(uint64_t sets, uint64_t points) {
  return align_up(8 * points, 256) + align_up(8 * (sets + 1), 256) + align_up(4 * points, 256) +
         align_up(4 * sets, 256) + chk::batch_layout((uint32_t)sets, points).total;
}

size_t slot_bytes_of(const ch_serve_config* cfg) {
  const int k = cfg->n_streams ? cfg->n_streams : kDefaultStreams;
  if (k < 1 || k > kMaxStreams) return 0;
  return cfg->arena_bytes / (size_t)k / 256 * 256;
}

uint64_t max_points_for_slot(size_t slot) {
  if (batch_need(1, 1) > slot) return 0;
  uint64_t lo = 1, hi = CH_MAX_POINTS;
  while (lo < hi) {  // largest n with batch_need(1, n) <= slot
    const uint64_t mid = lo + (hi - lo + 1) / 2;
    if (batch_need(1, mid) <= slot) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

struct Slot {
  ch_server* srv = nullptr;
  ch_ctx* ctx = nullptr;
  hipStream_t stream = nullptr;
  unsigned char* d_base = nullptr;
  unsigned char* pin_stage[2] = {nullptr, nullptr};  // kStageBytes each
  hipEvent_t stage_done[2] = {nullptr, nullptr};     // the last copy out of each
  uint64_t* pin_off = nullptr;                       // kMaxBatchSets + 1
  uint32_t* pin_cnt = nullptr;                       // kMaxBatchSets
  uint32_t* pin_hull = nullptr;                      // kPinHull
  std::thread th;
};

}  // namespace

struct ch_server {
  int device = 0;
  chs::Scheduler sched;
  std::vector<Slot> slots;
  explicit ch_server(chs::Config c) : sched(std::move(c)) {}
};

namespace {

void fail_all(std::vector<Request*>& b, ch_status st) {
  for (Request* r : b) {
    r->status = st;
    r->hull.clear();
  }
}

// Runs one batch on the slot's stream and fills every request's result.
void run_batch(Slot& sl, std::vector<Request*>& b) {
  // Small requests first (staged), then the rest, each set's offset in order.
  std::stable_partition(b.begin(), b.end(),
                        [](const Request* r) { return size_t(r->n) * 8 <= kStageReq; });
  const uint32_t nsets = (uint32_t)b.size();
  uint64_t total = 0;
  for (uint32_t i = 0; i < nsets; ++i) {
    sl.pin_off[i] = total;
    total += b[i]->n;
  }
  sl.pin_off[nsets] = total;

  unsigned char* p = sl.d_base;
  float* d_xy = reinterpret_cast<float*>(p);             p += align_up(8 * total, 256);
  uint64_t* d_off = reinterpret_cast<uint64_t*>(p);      p += align_up(8 * (uint64_t(nsets) + 1), 256);
  uint32_t* d_hidx = reinterpret_cast<uint32_t*>(p);     p += align_up(4 * total, 256);
  uint32_t* d_cnt = reinterpret_cast<uint32_t*>(p);      p += align_up(4 * uint64_t(nsets), 256);
  void* d_ws = p;
  const size_t ws_bytes = chk::batch_layout(nsets, total).total;

  hipStream_t st = sl.stream;
  hipError_t e = hipSuccess;
  // Staged copies: pack small requests into one staging buffer while the
  // other one's copy is in flight; a buffer is packed again only after the
  // event recorded behind its last copy has completed.
  int cur = 0;
  size_t staged = 0;
  bool fresh = true;  // the current buffer has not been waited for yet
  auto flush = [&](uint32_t first_set) {
    if (staged && e == hipSuccess) {
      e = hipMemcpyAsync(reinterpret_cast<unsigned char*>(d_xy) + 8 * sl.pin_off[first_set],
                         sl.pin_stage[cur], staged, hipMemcpyHostToDevice, st);
      if (e == hipSuccess) e = hipEventRecord(sl.stage_done[cur], st);
      cur ^= 1;
      fresh = true;
    }
    staged = 0;
  };
  uint32_t i = 0;
  uint32_t run_first = 0;
  for (; i < nsets && size_t(b[i]->n) * 8 <= kStageReq && e == hipSuccess; ++i) {
    const size_t bytes = size_t(b[i]->n) * 8;
    if (staged + bytes > kStageBytes) {
      flush(run_first);
      run_first = i;
    }
    if (fresh && bytes) {
      e = hipEventSynchronize(sl.stage_done[cur]);
      fresh = false;
    }
    if (bytes && e == hipSuccess) std::memcpy(sl.pin_stage[cur] + staged, b[i]->h_xy, bytes);
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
}

void worker(Slot* sl) {
  ch_server* s = sl->srv;
  (void)hipSetDevice(s->device);
  std::vector<Request*> b;
  while (s->sched.next_batch(b)) {
    run_batch(*sl, b);
    s->sched.finish(b);
  }
}

void destroy_slots(ch_server* s) {
  for (Slot& sl : s->slots) {
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
    if (sl.ctx) ch_ctx_destroy(sl.ctx);
    for (int k = 0; k < 2; ++k) {
      if (sl.pin_stage[k]) (void)hipHostFree(sl.pin_stage[k]);
      if (sl.stage_done[k]) (void)hipEventDestroy(sl.stage_done[k]);
    }
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
  // max_batch_points caps what several requests share; one request above it
  // still runs alone, so only the slot bounds a request.
  return max_points_for_slot(slot);
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
  chs::Config sc;
  sc.slot_bytes = slot;
  sc.max_req = ch_serve_max_request_points(cfg);
  sc.max_batch_points = cfg->max_batch_points;
  sc.max_inflight = cfg->max_inflight ? cfg->max_inflight : kDefaultInflight;
  sc.max_batch_sets = kMaxBatchSets;
  sc.need = batch_need;
  sc.now = now_ns;
  ch_server* s = new (std::nothrow) ch_server(std::move(sc));
  if (!s) return CH_E_NOMEM;
  s->device = dev;
  s->slots.resize(k);
  ch_status err = CH_OK;
  for (int i = 0; i < k && err == CH_OK; ++i) {
    Slot& sl = s->slots[i];
    sl.srv = s;
    sl.d_base = static_cast<unsigned char*>(cfg->d_arena) + size_t(i) * slot;
    if (ch_ctx_create(dev, nullptr, &sl.ctx) != CH_OK) { err = CH_E_DEVICE; break; }
    if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess) { err = CH_E_DEVICE; break; }
    for (int j = 0; j < 2 && err == CH_OK; ++j) {
      if (hipHostMalloc(reinterpret_cast<void**>(&sl.pin_stage[j]), kStageBytes, hipHostMallocDefault) !=
          hipSuccess)
        err = CH_E_NOMEM;
      else if (hipEventCreateWithFlags(&sl.stage_done[j], hipEventDisableTiming) != hipSuccess)
        err = CH_E_DEVICE;
    }
    if (err != CH_OK) break;
    if (hipHostMalloc(reinterpret_cast<void**>(&sl.pin_off), 8 * (size_t(kMaxBatchSets) + 1),
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
  if (!s) return CH_E_INVALID_ARG;
  return s->sched.submit(h_xy, n, ticket);
}

ch_status ch_serve_wait(ch_server* s, uint64_t ticket, int64_t timeout_us, uint32_t* hull_idx,
                        uint32_t cap, uint32_t* h_out, uint64_t* t_ns) {
  if (!s) return CH_E_INVALID_ARG;
  return s->sched.wait(ticket, timeout_us, hull_idx, cap, h_out, t_ns);
}

ch_status ch_serve_stats(ch_server* s, uint64_t* completed, uint64_t* batches, double* hulls_per_s,
                         double* p50_us, double* p99_us) {
  if (!s) return CH_E_INVALID_ARG;
  s->sched.stats(completed, batches, hulls_per_s, p50_us, p99_us);
  return CH_OK;
}

ch_status ch_serve_stop(ch_server* s) {
  if (!s) return CH_E_INVALID_ARG;
  s->sched.stop_begin();
  for (Slot& sl : s->slots)
    if (sl.th.joinable()) sl.th.join();
  s->sched.stop_finish();
  destroy_slots(s);
  delete s;
  return CH_OK;
}

}  // extern "C"
