// Host-side scheduling of the request server (ch_serve_*): the request queue,
// tickets, continuous batching under the slot budget, completion, waits and
// latency statistics. No HIP here: a worker takes a batch with next_batch(),
// runs it on the device itself, and hands it back with finish(). Kept apart
// from the device code so that it can be unit-tested on the CPU with a fake
// executor and clock (and a thread sanitizer).
#pragma once

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdint>
#include <cstring>
#include <deque>
#include <functional>
#include <mutex>
#include <new>
#include <unordered_map>
#include <vector>

#include "../../include/convhull.h"

namespace chs {

struct Request {
  const float* h_xy = nullptr;
  uint32_t n = 0;
  ch_status status = CH_OK;
  bool done = false;
  bool waiting = false;
  std::vector<uint32_t> hull;
  uint64_t t_arrive = 0, t_admit = 0, t_done = 0;
};

// Completion latencies in a fixed log-linear histogram: 32 buckets per
// power of two of nanoseconds (relative width 2.2 %), so the statistics of
// any number of requests take constant memory. A percentile reports the
// geometric middle of its bucket (within 1.1 % of the exact order
// statistic).
class LatencyHistogram {
 public:
  static constexpr int kSub = 32;
  static constexpr int kBuckets = 64 * kSub;
  void add(uint64_t ns) {
    counts_[bucket(ns)] += 1;
    total_ += 1;
  }
  uint64_t total() const { return total_; }
  // Nearest-rank percentile q in (0, 100], in microseconds (0 when empty).
  double percentile_us(double q) const {
    if (!total_) return 0.0;
    uint64_t rank = (uint64_t)std::ceil(q / 100.0 * double(total_));
    if (rank < 1) rank = 1;
    uint64_t seen = 0;
    for (int b = 0; b < kBuckets; ++b) {
      seen += counts_[b];
      if (seen >= rank) return mid_ns(b) * 1e-3;
    }
    return mid_ns(kBuckets - 1) * 1e-3;
  }
  static int bucket(uint64_t ns) {
    if (ns < 2) return 0;
    const int e = 63 - __builtin_clzll(ns);  // 2^e <= ns < 2^(e+1)
    const double f = double(ns) / double(1ull << e);  // [1, 2)
    int s = (int)(std::log2(f) * kSub);
    if (s >= kSub) s = kSub - 1;
    return e * kSub + s;
  }
  static double mid_ns(int b) {
    const int e = b / kSub, s = b % kSub;
    return std::exp2(double(e) + (double(s) + 0.5) / kSub);
  }

 private:
  uint64_t counts_[kBuckets] = {};
  uint64_t total_ = 0;
};

struct Config {
  size_t slot_bytes = 0;          // device budget of one batch
  uint64_t max_req = 0;           // largest request (points)
  uint64_t max_batch_points = 0;  // 0: no cap beyond the budget
  uint32_t max_inflight = 65536;
  uint32_t max_batch_sets = 65536;
  // Device bytes a batch of `sets` requests with `points` points needs.
  std::function<size_t(uint64_t sets, uint64_t points)> need;
  // Steady-clock nanoseconds.
  std::function<uint64_t()> now;
};

class Scheduler {
 public:
  explicit Scheduler(Config cfg) : cfg_(std::move(cfg)) {}
  ~Scheduler() {
    for (auto& kv : tickets_) delete kv.second;
  }
  const Config& config() const { return cfg_; }

  // Queue one request. CH_E_INVALID_ARG (too large, null data), CH_E_BUSY
  // (max_inflight outstanding), CH_E_SHUTDOWN (stopping), CH_E_NOMEM.
  ch_status submit(const float* h_xy, uint32_t n, uint64_t* ticket) {
    if (!ticket || (n && !h_xy)) return CH_E_INVALID_ARG;
    if (n > cfg_.max_req) return CH_E_INVALID_ARG;
    Request* r = new (std::nothrow) Request();
    if (!r) return CH_E_NOMEM;
    r->h_xy = h_xy;
    r->n = n;
    r->t_arrive = cfg_.now();
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (stopping_) {
        delete r;
        return CH_E_SHUTDOWN;
      }
      if (inflight_ >= cfg_.max_inflight) {
        delete r;
        return CH_E_BUSY;
      }
      const uint64_t t = next_ticket_++;
      tickets_.emplace(t, r);
      queue_.push_back(r);
      inflight_ += 1;
      *ticket = t;
    }
    cv_work_.notify_one();
    return CH_OK;
  }

  // Worker side: blocks until requests are queued (returns them as one batch,
  // in arrival order, as many as fit the budget and the point cap; at least
  // one) or the scheduler stops (returns false).
  bool next_batch(std::vector<Request*>& b) {
    b.clear();
    std::unique_lock<std::mutex> lk(mu_);
    cv_work_.wait(lk, [&] { return stopping_ || !queue_.empty(); });
    if (stopping_) return false;
    uint64_t pts = 0;
    while (!queue_.empty() && b.size() < cfg_.max_batch_sets) {
      Request* r = queue_.front();
      const uint64_t p2 = pts + r->n;
      if (!b.empty()) {
        if (cfg_.need(b.size() + 1, p2) > cfg_.slot_bytes) break;
        if (cfg_.max_batch_points && p2 > cfg_.max_batch_points) break;
      }
      b.push_back(r);
      queue_.pop_front();
      pts = p2;
    }
    const uint64_t t = cfg_.now();
    for (Request* r : b) r->t_admit = t;
    return true;
  }

  // Worker side: the batch's results are in its requests (status, hull).
  void finish(const std::vector<Request*>& b) {
    const uint64_t t = cfg_.now();
    std::lock_guard<std::mutex> lk(mu_);
    for (Request* r : b) {
      r->t_done = t;
      r->done = true;
      completed_ += 1;
      lat_.add(t - r->t_arrive);
      if (!first_arrive_ || r->t_arrive < first_arrive_) first_arrive_ = r->t_arrive;
    }
    last_done_ = t;
    batches_ += 1;
    cv_done_.notify_all();
  }

  ch_status wait(uint64_t ticket, int64_t timeout_us, uint32_t* hull_idx, uint32_t cap,
                 uint32_t* h_out, uint64_t* t_ns) {
    if (!h_out || (cap && !hull_idx)) return CH_E_INVALID_ARG;
    std::unique_lock<std::mutex> lk(mu_);
    auto it = tickets_.find(ticket);
    if (it == tickets_.end()) return CH_E_NOT_FOUND;
    Request* r = it->second;
    if (r->waiting) return CH_E_INVALID_ARG;
    r->waiting = true;
    active_waiters_ += 1;
    auto leave = [&](ch_status st) {
      active_waiters_ -= 1;
      cv_done_.notify_all();
      return st;
    };
    if (timeout_us < 0) {
      cv_done_.wait(lk, [&] { return r->done; });
    } else {
      cv_done_.wait_for(lk, std::chrono::microseconds(timeout_us), [&] { return r->done; });
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
    tickets_.erase(it);
    inflight_ -= 1;
    delete r;
    return leave(st);
  }

  void stats(uint64_t* completed, uint64_t* batches, double* hulls_per_s, double* p50_us,
             double* p99_us) {
    std::lock_guard<std::mutex> lk(mu_);
    if (completed) *completed = completed_;
    if (batches) *batches = batches_;
    if (hulls_per_s)
      *hulls_per_s = (completed_ && last_done_ > first_arrive_)
                         ? double(completed_) / (double(last_done_ - first_arrive_) * 1e-9)
                         : 0.0;
    if (p50_us) *p50_us = lat_.percentile_us(50.0);
    if (p99_us) *p99_us = lat_.percentile_us(99.0);
  }

  // Stop, first half: refuse new submissions, resolve every queued request
  // that was never admitted with CH_E_SHUTDOWN, and wake the workers
  // (next_batch returns false; batches already taken still finish).
  void stop_begin() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stopping_ = true;
      const uint64_t t = cfg_.now();
      for (Request* r : queue_) {
        r->status = CH_E_SHUTDOWN;
        r->t_done = t;
        r->done = true;
      }
      queue_.clear();
    }
    cv_work_.notify_all();
    cv_done_.notify_all();
  }

  // Stop, second half (after the workers have exited): wake blocked waiters
  // and wait until every one of them has returned.
  void stop_finish() {
    std::unique_lock<std::mutex> lk(mu_);
    cv_done_.notify_all();
    cv_done_.wait(lk, [&] { return active_waiters_ == 0; });
  }

 private:
  Config cfg_;
  std::mutex mu_;
  std::condition_variable cv_work_;  // queue or stop
  std::condition_variable cv_done_;  // a request finished, a waiter left
  std::deque<Request*> queue_;
  std::unordered_map<uint64_t, Request*> tickets_;
  uint64_t next_ticket_ = 1;
  uint32_t inflight_ = 0;
  bool stopping_ = false;
  int active_waiters_ = 0;
  uint64_t completed_ = 0, batches_ = 0;
  uint64_t first_arrive_ = 0, last_done_ = 0;
  LatencyHistogram lat_;
};

}  // namespace chs
