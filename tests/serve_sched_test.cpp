// Host test of the uplift server's scheduler policy (admission by budget,
// first come first served, same-key merging, continuous admission,
// cancellation of waiting requests, failure isolation of merged passes),
// with a stand-in executor instead of the GPU.  Built and run by
// test_serve_sched.py, also under ThreadSanitizer.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <thread>
#include <vector>

#include "serve_sched.h"

struct Req {
  int64_t bytes;
  int32_t D;
  uint64_t key;
  int id;
};

#define CHECK(c)                                                     \
  do {                                                               \
    if (!(c)) {                                                      \
      std::fprintf(stderr, "FAILED line %d: %s\n", __LINE__, #c);    \
      std::exit(1);                                                  \
    }                                                                \
  } while (0)

static std::vector<int> ids(const std::vector<Req>& b) {
  std::vector<int> v;
  for (const Req& r : b) v.push_back(r.id);
  return v;
}

int main() {
  std::vector<Req> b;
  {  // the admission hook sees requests in admission order, when the budget allows
    std::vector<int> order;
    lv::Scheduler<Req> s(100, 8, 1024, [&](Req& r) { order.push_back(r.id); });
    CHECK(s.submit({60, 1, 1, 1}));
    CHECK(s.submit({50, 1, 2, 2}));
    CHECK(s.submit({30, 1, 3, 3}));
    CHECK(order == std::vector<int>({1}));
    CHECK(s.next_batch(b) && ids(b) == std::vector<int>({1}));
    s.complete(b);
    CHECK(order == std::vector<int>({1, 2, 3}));
    CHECK(s.next_batch(b));
    s.complete(b);
    CHECK(s.next_batch(b));
    s.complete(b);
  }
  {  // refusal, FIFO admission blocking behind a request that does not fit
    lv::Scheduler<Req> s(100, 8, 1024);
    CHECK(!s.submit({101, 1, 1, 0}));
    CHECK(s.submit({60, 1, 1, 1}));
    CHECK(s.submit({50, 1, 2, 2}));
    CHECK(s.submit({30, 1, 3, 3}));  // would fit, but waits behind request 2
    CHECK(s.used() == 60);
    CHECK(s.next_batch(b) && ids(b) == std::vector<int>({1}));
    s.complete(b);  // frees 60: requests 2 and 3 are admitted together
    CHECK(s.used() == 80);
    CHECK(s.next_batch(b) && ids(b) == std::vector<int>({2}));
    CHECK(s.next_batch(b) && ids(b) == std::vector<int>({3}));
    CHECK(s.peak_used() == 80);
  }
  {  // merging: same key, oldest first, at most max_sets
    lv::Scheduler<Req> s(1000, 2, 1024);
    s.submit({1, 8, 7, 0});
    s.submit({1, 8, 9, 1});
    s.submit({1, 8, 7, 2});
    s.submit({1, 8, 7, 3});
    CHECK(s.next_batch(b) && ids(b) == std::vector<int>({0, 2}));
    CHECK(s.next_batch(b) && ids(b) == std::vector<int>({1}));
    CHECK(s.next_batch(b) && ids(b) == std::vector<int>({3}));
  }
  {  // channel cap
    lv::Scheduler<Req> s(1000, 8, 100);
    s.submit({1, 64, 7, 0});
    s.submit({1, 64, 7, 1});
    s.submit({1, 30, 7, 2});
    CHECK(s.next_batch(b) && ids(b) == std::vector<int>({0, 2}));
    CHECK(s.next_batch(b) && ids(b) == std::vector<int>({1}));
  }
  {  // cancellation: a pending request (blocking the queue) and an admitted one
    lv::Scheduler<Req> s(100, 8, 1024);
    CHECK(s.submit({60, 1, 1, 0}));
    CHECK(s.submit({50, 1, 2, 1}));   // pending: 60 + 50 > 100
    CHECK(s.submit({30, 1, 3, 2}));   // pending behind request 1
    Req out{};
    CHECK(s.cancel([](const Req& r) { return r.id == 1; }, &out) && out.id == 1);
    CHECK(s.used() == 90);            // request 2 admitted once 1 no longer blocks it
    CHECK(s.cancel([](const Req& r) { return r.id == 2; }, &out) && out.id == 2);
    CHECK(s.used() == 60);            // an admitted request's memory returns
    CHECK(!s.cancel([](const Req& r) { return r.id == 7; }, &out));
    CHECK(s.next_batch(b) && ids(b) == std::vector<int>({0}));
    CHECK(!s.cancel([](const Req& r) { return r.id == 0; }, &out));  // running
    s.complete(b);
    s.drain();                        // cancelled requests no longer count as outstanding
    CHECK(s.used() == 0);
  }
  {  // failure isolation: a failing merged pass runs each request alone
    std::vector<std::vector<size_t>> calls;
    auto run = [&](const std::vector<size_t>& idx) {
      calls.push_back(idx);
      for (size_t k : idx)
        if (k == 1) return 2;         // request 1 is malformed
      return 0;
    };
    std::vector<int> st = lv::run_isolated(3, 3, run);
    CHECK(st == std::vector<int>({0, 2, 0}));
    CHECK(calls.size() == 4 && calls[0].size() == 3);
    calls.clear();
    auto fatal = [&](const std::vector<size_t>& idx) {
      calls.push_back(idx);
      return 3;                       // a device fault: no reruns
    };
    CHECK(lv::run_isolated(3, 3, fatal) == std::vector<int>({3, 3, 3}) && calls.size() == 1);
    calls.clear();
    CHECK(lv::run_isolated(2, 3, run) == std::vector<int>({0, 2}) && calls.size() == 3);
  }
  {  // concurrent workers, random arrivals: budget never exceeded, every
     // request served exactly once, batches homogeneous and within limits
    const int64_t budget = 1000;
    const int max_sets = 3, max_ch = 200, nreq = 400, nworkers = 4;
    lv::Scheduler<Req> s(budget, max_sets, max_ch);
    std::atomic<int64_t> live_bytes{0}, max_live{0};
    std::vector<std::atomic<int>> served(nreq);
    for (auto& x : served) x = 0;
    std::atomic<int> passes{0}, merged{0};
    std::vector<std::thread> ws;
    for (int w = 0; w < nworkers; w++) {
      ws.emplace_back([&, w] {
        std::mt19937 rng(w);
        std::vector<Req> batch;
        while (s.next_batch(batch)) {
          int64_t bytes = 0;
          int ch = 0;
          for (const Req& r : batch) {
            bytes += r.bytes;
            ch += r.D;
            CHECK(r.key == batch[0].key);
            served[r.id]++;
          }
          CHECK((int)batch.size() <= max_sets);
          CHECK(ch <= max_ch || batch.size() == 1);
          const int64_t now = live_bytes += bytes;
          int64_t prev = max_live;
          while (now > prev && !max_live.compare_exchange_weak(prev, now)) {
          }
          std::this_thread::sleep_for(std::chrono::microseconds(50 + rng() % 200));
          live_bytes -= bytes;
          passes++;
          if (batch.size() > 1) merged++;
          s.complete(batch);
        }
      });
    }
    std::mt19937 rng(42);
    std::vector<int> cancelled;
    for (int i = 0; i < nreq; i++) {
      Req r{(int64_t)(1 + rng() % 400), (int32_t)(1 + rng() % 128), (uint64_t)(rng() % 3), i};
      CHECK(s.submit(r));
      if (rng() % 4 == 0) std::this_thread::sleep_for(std::chrono::microseconds(rng() % 100));
      if (i > 10 && rng() % 8 == 0) {  // cancel an earlier request if it is still waiting
        const int victim = i - 1 - (int)(rng() % 10);
        Req out{};
        if (s.cancel([victim](const Req& q) { return q.id == victim; }, &out)) cancelled.push_back(victim);
      }
    }
    s.drain();
    CHECK(s.used() == 0);
    s.shutdown();
    for (auto& t : ws) t.join();
    for (int v : cancelled) CHECK(served[v] == 0);
    for (int i = 0; i < nreq; i++)
      CHECK(served[i] == (std::find(cancelled.begin(), cancelled.end(), i) == cancelled.end() ? 1 : 0));
    CHECK(max_live <= budget);
    CHECK(s.peak_used() <= budget);
    CHECK(merged > 0);
    std::printf("ok passes=%d merged=%d cancelled=%d peak=%lld\n", passes.load(), merged.load(),
                (int)cancelled.size(), (long long)s.peak_used());
  }
  return 0;
}
