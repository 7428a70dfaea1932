// Host test of the uplift server's scheduler policy (admission by budget,
// first come first served, same-key merging, continuous admission), with a
// stand-in executor instead of the GPU.  Built and run by test_serve_sched.py.
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
    for (int i = 0; i < nreq; i++) {
      Req r{(int64_t)(1 + rng() % 400), (int32_t)(1 + rng() % 128), (uint64_t)(rng() % 3), i};
      CHECK(s.submit(r));
      if (rng() % 4 == 0) std::this_thread::sleep_for(std::chrono::microseconds(rng() % 100));
    }
    s.drain();
    CHECK(s.used() == 0);
    s.shutdown();
    for (auto& t : ws) t.join();
    for (int i = 0; i < nreq; i++) CHECK(served[i] == 1);
    CHECK(max_live <= budget);
    CHECK(s.peak_used() <= budget);
    CHECK(merged > 0);
    std::printf("ok passes=%d merged=%d peak=%lld\n", passes.load(), merged.load(),
                (long long)s.peak_used());
  }
  return 0;
}
