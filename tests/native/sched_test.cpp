// CPU unit test of the request server's scheduler (ch_sched.hpp) with a fake
// executor and a fake clock: admission under the slot budget, arrival
// order, the point and set caps, back-pressure, time-outs, capacity retries, per-ticket failure
// statuses injected by the executor, shutdown, the latency percentiles, and
// many submitting / waiting / working threads at once (built with a thread
// sanitizer by tests/test_serve_scheduler.py). Prints "ok" and exits 0 when
// every check holds.
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <thread>
#include <vector>

#include "ch_sched.hpp"

namespace {

int g_fail = 0;
#define CHECK(c)                                                        \
  do {                                                                  \
    if (!(c)) {                                                         \
      std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
      ++g_fail;                                                         \
    }                                                                   \
  } while (0)

std::atomic<uint64_t> g_clock{1};
uint64_t fake_now() { return g_clock.load(); }

// Budget: 100 bytes per set plus 10 per point.
size_t fake_need(uint64_t sets, uint64_t points) { return size_t(100 * sets + 10 * points); }

chs::Config make_cfg(size_t slot, uint32_t inflight = 1000) {
  chs::Config c;
  c.slot_bytes = slot;
  c.max_req = 5000;
  c.max_inflight = inflight;
  c.need = fake_need;
  c.now = fake_now;
  return c;
}

// The fake device: every request's "hull" is (n, its first coordinate's
// bits); a request of 13 points makes the whole batch fail with
// CH_E_DEVICE, one of 17 points fails alone with CH_E_NOMEM.
void execute(std::vector<chs::Request*>& b) {
  bool poison = false;
  for (auto* r : b) poison |= r->n == 13;
  for (auto* r : b) {
    if (poison) {
      r->status = CH_E_DEVICE;
      r->hull.clear();
    } else if (r->n == 17) {
      r->status = CH_E_NOMEM;
    } else {
      uint32_t bits = 0;
      if (r->n) std::memcpy(&bits, r->h_xy, 4);
      r->status = CH_OK;
      r->hull = {r->n, bits};
    }
  }
}

void test_batching_budget_and_order() {
  chs::Scheduler s(make_cfg(5000));
  std::vector<float> data(5000, 0.5f);
  std::vector<uint64_t> t;
  const uint32_t sizes[] = {100, 200, 300, 50, 400, 10, 4000, 5, 5};
  for (uint32_t n : sizes) {
    uint64_t k = 0;
    CHECK(s.submit(data.data(), n, &k) == CH_OK);
    t.push_back(k);
  }
  std::vector<chs::Request*> b;
  std::vector<uint32_t> order;
  int batches = 0;
  size_t left = sizeof(sizes) / sizeof(sizes[0]);
  while (left) {
    CHECK(s.next_batch(b));
    CHECK(!b.empty());
    uint64_t pts = 0;
    for (auto* r : b) { pts += r->n; order.push_back(r->n); }
    // Every batch of more than one request fits the budget.
    if (b.size() > 1) CHECK(fake_need(b.size(), pts) <= 5000);
    execute(b);
    s.finish(b);
    left -= b.size();
    ++batches;
  }
  CHECK(batches >= 2);
  // Arrival order is kept across batches.
  for (size_t i = 0; i < order.size(); ++i) CHECK(order[i] == sizes[i]);
  for (size_t i = 0; i < t.size(); ++i) {
    uint32_t hull[2], h = 0;
    uint64_t tn[3];
    CHECK(s.wait(t[i], 0, hull, 2, &h, tn) == CH_OK);
    CHECK(h == 2 && hull[0] == sizes[i]);
    CHECK(tn[0] <= tn[1] && tn[1] <= tn[2]);
  }
  uint64_t done = 0, nb = 0;
  s.stats(&done, &nb, nullptr, nullptr, nullptr);
  CHECK(done == t.size() && nb == (uint64_t)batches);
}

// The point cap (max_batch_points) and the set cap (max_batch_sets): a
// batch of several requests stays within both, a request above the point
// cap runs alone, and arrival order holds across batches.
void test_batch_point_and_set_caps() {
  chs::Config c = make_cfg(1u << 30);
  c.max_batch_points = 500;
  c.max_batch_sets = 3;
  chs::Scheduler s(c);
  std::vector<float> data(5000, 0.25f);
  const uint32_t sizes[] = {100, 100, 100, 100, 900, 10, 10, 480, 30, 1, 1, 1, 1};
  std::vector<uint64_t> t;
  for (uint32_t n : sizes) {
    uint64_t k = 0;
    CHECK(s.submit(data.data(), n, &k) == CH_OK);
    t.push_back(k);
  }
  std::vector<chs::Request*> b;
  std::vector<uint32_t> order;
  std::vector<size_t> lens;
  size_t left = sizeof(sizes) / sizeof(sizes[0]);
  while (left) {
    CHECK(s.next_batch(b));
    CHECK(!b.empty() && b.size() <= 3);
    uint64_t pts = 0;
    for (auto* r : b) { pts += r->n; order.push_back(r->n); }
    if (b.size() > 1) CHECK(pts <= 500);
    lens.push_back(b.size());
    execute(b);
    s.finish(b);
    left -= b.size();
  }
  for (size_t i = 0; i < order.size(); ++i) CHECK(order[i] == sizes[i]);
  // Greedy in arrival order: {100,100,100} (set cap), {100} (900 would pass
  // the point cap), {900} alone, {10,10,480}, {30,1,1} (set cap), {1,1}.
  const size_t want[] = {3, 1, 1, 3, 3, 2};
  CHECK(lens.size() == sizeof(want) / sizeof(want[0]));
  for (size_t i = 0; i < lens.size() && i < sizeof(want) / sizeof(want[0]); ++i) CHECK(lens[i] == want[i]);
  for (size_t i = 0; i < t.size(); ++i) {
    uint32_t hull[2], h = 0;
    CHECK(s.wait(t[i], 0, hull, 2, &h, nullptr) == CH_OK);
    CHECK(h == 2 && hull[0] == sizes[i]);
  }
}

void test_admission_errors_and_backpressure() {
  chs::Scheduler s(make_cfg(100000, 3));
  std::vector<float> data(6000, 0.25f);
  uint64_t k = 0;
  CHECK(s.submit(data.data(), 5001, &k) == CH_E_INVALID_ARG);  // above max_req
  CHECK(s.submit(nullptr, 4, &k) == CH_E_INVALID_ARG);
  CHECK(s.submit(data.data(), 4, nullptr) == CH_E_INVALID_ARG);
  uint64_t a, b2, c, d;
  CHECK(s.submit(data.data(), 4, &a) == CH_OK);
  CHECK(s.submit(data.data(), 5, &b2) == CH_OK);
  CHECK(s.submit(nullptr, 0, &c) == CH_OK);  // an empty request needs no data
  CHECK(s.submit(data.data(), 6, &d) == CH_E_BUSY);
  std::vector<chs::Request*> b;
  CHECK(s.next_batch(b) && b.size() == 3);
  execute(b);
  s.finish(b);
  uint32_t hull[2], h = 0;
  CHECK(s.wait(a, -1, hull, 2, &h, nullptr) == CH_OK);
  CHECK(s.wait(a, -1, hull, 2, &h, nullptr) == CH_E_NOT_FOUND);
  CHECK(s.wait(999, 0, hull, 2, &h, nullptr) == CH_E_NOT_FOUND);
  CHECK(s.submit(data.data(), 6, &d) == CH_OK);  // room again
  // Capacity: the ticket is kept, a larger buffer collects it.
  CHECK(s.wait(b2, -1, hull, 1, &h, nullptr) == CH_E_CAPACITY && h == 2);
  CHECK(s.wait(b2, -1, hull, 2, &h, nullptr) == CH_OK && hull[0] == 5);
  CHECK(s.wait(c, -1, hull, 2, &h, nullptr) == CH_OK && h == 2 && hull[0] == 0);
  // Time-out: d is queued and no worker runs; the ticket stays valid.
  CHECK(s.wait(d, 1000, hull, 2, &h, nullptr) == CH_E_TIMEOUT);
  CHECK(s.next_batch(b) && b.size() == 1);
  execute(b);
  s.finish(b);
  CHECK(s.wait(d, 0, hull, 2, &h, nullptr) == CH_OK && hull[0] == 6);
}

void test_injected_failures_per_ticket() {
  chs::Scheduler s(make_cfg(1000000));
  std::vector<float> data(100, 0.75f);
  uint64_t t1, t2, t3, t4;
  CHECK(s.submit(data.data(), 17, &t1) == CH_OK);  // fails alone (CH_E_NOMEM)
  CHECK(s.submit(data.data(), 20, &t2) == CH_OK);
  std::vector<chs::Request*> b;
  CHECK(s.next_batch(b) && b.size() == 2);
  execute(b);
  s.finish(b);
  CHECK(s.submit(data.data(), 13, &t3) == CH_OK);  // poisons its batch (CH_E_DEVICE)
  CHECK(s.submit(data.data(), 30, &t4) == CH_OK);
  CHECK(s.next_batch(b) && b.size() == 2);
  execute(b);
  s.finish(b);
  uint32_t hull[2], h = 0;
  CHECK(s.wait(t1, -1, hull, 2, &h, nullptr) == CH_E_NOMEM);
  CHECK(s.wait(t2, -1, hull, 2, &h, nullptr) == CH_OK && hull[0] == 20);
  CHECK(s.wait(t3, -1, hull, 2, &h, nullptr) == CH_E_DEVICE);
  CHECK(s.wait(t4, -1, hull, 2, &h, nullptr) == CH_E_DEVICE);
  // Failed tickets are released like successful ones.
  CHECK(s.wait(t3, 0, hull, 2, &h, nullptr) == CH_E_NOT_FOUND);
}

void test_percentiles_with_a_fake_clock() {
  chs::Scheduler s(make_cfg(1000000));
  std::vector<float> data(4, 0.5f);
  std::vector<chs::Request*> b;
  std::vector<uint64_t> tk;
  // Request i arrives at 10 ms * i and completes (i + 1) microseconds later.
  for (int i = 0; i < 1000; ++i) {
    g_clock = 10000000ull * (i + 1);
    uint64_t k;
    CHECK(s.submit(data.data(), 4, &k) == CH_OK);
    tk.push_back(k);
    CHECK(s.next_batch(b) && b.size() == 1);
    execute(b);
    g_clock = 10000000ull * (i + 1) + 1000ull * (i + 1);
    s.finish(b);
  }
  double p50 = 0, p99 = 0, rate = 0;
  uint64_t done = 0;
  s.stats(&done, nullptr, &rate, &p50, &p99);
  CHECK(done == 1000);
  // Nearest rank: 500 us and 990 us, within the histogram's 1.1 %.
  CHECK(std::fabs(p50 - 500.0) / 500.0 < 0.012);
  CHECK(std::fabs(p99 - 990.0) / 990.0 < 0.012);
  // 1000 requests from the first arrival (10 ms) to the last completion.
  const double span = (10000000.0 * 1000 + 1000.0 * 1000 - 10000000.0) * 1e-9;
  CHECK(std::fabs(rate - 1000.0 / span) / (1000.0 / span) < 1e-9);
  uint32_t hull[2], h;
  for (uint64_t k : tk) CHECK(s.wait(k, 0, hull, 2, &h, nullptr) == CH_OK);
}

void test_stop_resolves_queue_and_wakes_waiters() {
  chs::Scheduler s(make_cfg(100 + 10 * 10));  // one 10-point request per batch
  std::vector<float> data(10, 0.5f);
  std::vector<uint64_t> tk(6);
  for (auto& k : tk) CHECK(s.submit(data.data(), 10, &k) == CH_OK);
  std::vector<chs::Request*> held;
  CHECK(s.next_batch(held) && held.size() == 1);  // admitted, not finished
  std::atomic<int> got_last{-1};
  std::thread waiter([&] {
    uint32_t hull[2], h;
    got_last = (int)s.wait(tk.back(), -1, hull, 2, &h, nullptr);
  });
  std::thread worker_exit([&] {
    std::vector<chs::Request*> b;
    // Blocks until stop: nothing else is taken once stop has begun... or
    // takes queued work first; either way every request gets a final status.
    while (s.next_batch(b)) {
      execute(b);
      s.finish(b);
    }
  });
  std::this_thread::sleep_for(std::chrono::milliseconds(20));
  s.stop_begin();
  worker_exit.join();
  execute(held);
  s.finish(held);  // the admitted batch still completes
  s.stop_finish();
  waiter.join();
  CHECK(got_last == (int)CH_E_SHUTDOWN || got_last == (int)CH_OK);
  uint32_t hull[2], h;
  CHECK(s.wait(tk[0], 0, hull, 2, &h, nullptr) == CH_OK && hull[0] == 10);
  uint64_t k;
  CHECK(s.submit(data.data(), 10, &k) == CH_E_SHUTDOWN);
  for (size_t i = 1; i + 1 < tk.size(); ++i) {
    const ch_status st = s.wait(tk[i], 0, hull, 2, &h, nullptr);
    CHECK(st == CH_E_SHUTDOWN || st == CH_OK);
  }
}

void test_many_threads() {
  chs::Config c = make_cfg(100 * 64 + 10 * 4096, 100000);
  c.now = [] {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
  };
  chs::Scheduler s(std::move(c));
  constexpr int kSubmitters = 6, kPer = 1500, kWorkers = 3;
  std::vector<std::vector<float>> data(kSubmitters);
  for (int i = 0; i < kSubmitters; ++i) data[i].assign(64, float(i) * 0.125f);
  std::vector<std::thread> workers;
  for (int w = 0; w < kWorkers; ++w)
    workers.emplace_back([&] {
      std::vector<chs::Request*> b;
      while (s.next_batch(b)) {
        execute(b);
        s.finish(b);
      }
    });
  std::atomic<int> bad{0};
  std::atomic<bool> polling{true};
  std::thread poller([&] {  // statistics read while requests complete
    while (polling) {
      uint64_t d = 0;
      double a = 0, b = 0, r = 0;
      s.stats(&d, nullptr, &r, &a, &b);
      if (a > b) ++bad;
      std::this_thread::yield();
    }
  });
  std::vector<std::thread> subs;
  for (int i = 0; i < kSubmitters; ++i)
    subs.emplace_back([&, i] {
      std::vector<uint64_t> mine;
      for (int j = 0; j < kPer; ++j) {
        const uint32_t n = 1 + (uint32_t)((i * 7 + j) % 60);
        uint64_t k;
        ch_status st;
        while ((st = s.submit(data[i].data(), n == 13 || n == 17 ? 12 : n, &k)) == CH_E_BUSY)
          std::this_thread::yield();
        if (st != CH_OK) { ++bad; continue; }
        mine.push_back(k);
        if (mine.size() > 64) {  // collect in arrival order as we go
          uint32_t hull[2], h;
          if (s.wait(mine.front(), -1, hull, 2, &h, nullptr) != CH_OK) ++bad;
          uint32_t want;
          std::memcpy(&want, data[i].data(), 4);
          if (hull[1] != want) ++bad;
          mine.erase(mine.begin());
        }
      }
      for (uint64_t k : mine) {
        uint32_t hull[2], h;
        if (s.wait(k, -1, hull, 2, &h, nullptr) != CH_OK) ++bad;
      }
    });
  for (auto& t : subs) t.join();
  polling = false;
  poller.join();
  uint64_t done = 0;
  double p50 = 0, p99 = 0;
  s.stats(&done, nullptr, nullptr, &p50, &p99);
  s.stop_begin();
  for (auto& t : workers) t.join();
  s.stop_finish();
  CHECK(bad == 0);
  CHECK(done == (uint64_t)kSubmitters * kPer);
  CHECK(p50 > 0 && p50 <= p99);
}

void test_histogram() {
  using H = chs::LatencyHistogram;
  // Buckets are monotone and every value lies within its bucket's 2.2 %.
  int prev = -1;
  for (uint64_t v = 1; v < (1ull << 40); v = v + v / 7 + 1) {
    const int b = H::bucket(v);
    CHECK(b >= prev);
    prev = b;
    if (v >= 64) CHECK(std::fabs(H::mid_ns(b) - double(v)) / double(v) < 0.0225);
  }
  H h;
  CHECK(h.percentile_us(50) == 0.0);
}

}  // namespace

int main() {
  test_histogram();
  test_batching_budget_and_order();
  test_batch_point_and_set_caps();
  test_admission_errors_and_backpressure();
  test_injected_failures_per_ticket();
  test_percentiles_with_a_fake_clock();
  test_stop_resolves_queue_and_wakes_waiters();
  test_many_threads();
  if (g_fail) {
    std::fprintf(stderr, "%d check(s) failed\n", g_fail);
    return 1;
  }
  std::printf("ok\n");
  return 0;
}
