// Request scheduler of the uplift server: admission by a memory budget and
// same-scene batching, independent of the GPU (plain C++17, so that its
// policy can be exercised on the host with a stand-in executor).
//
// Policy:
//   * Admission is first come, first served: the oldest pending request is
//     admitted as soon as its working memory fits in what the budget has
//     left; a request that does not fit blocks those behind it (no
//     starvation of large requests).  A request larger than the whole budget
//     is refused at submission.
//   * A free worker takes the oldest admitted request and merges into the
//     same pass every other admitted request with the same batch key (scene
//     and storage dtype), oldest first, while the pass has at most
//     `max_sets` requests and `max_channels` channels.
//   * A finished pass returns its requests' memory to the budget, which may
//     admit more requests while other passes are still running: requests
//     join as slots and memory free up (continuous batching across passes).
//   * A waiting request (pending or admitted, not yet in a pass) can be
//     cancelled; its memory returns to the budget.
//   * A merged pass that fails with a request-level error runs each of its
//     requests again alone (run_isolated), so that one malformed request
//     does not fail the others.
#pragma once

#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <mutex>
#include <functional>
#include <vector>

namespace lv {

template <typename Req>
class Scheduler {
 public:
  // Req must provide: int64_t bytes; int32_t D; uint64_t key; and is moved.
  // on_admit (optional) sees each request as it is admitted, in admission
  // order, under the scheduler's lock.
  Scheduler(int64_t budget, int max_sets, int max_channels,
            std::function<void(Req&)> on_admit = std::function<void(Req&)>())
      : budget_(budget), max_sets_(max_sets), max_channels_(max_channels), on_admit_(std::move(on_admit)) {}

  // false: the request can never be admitted (larger than the budget)
  bool submit(Req r) {
    if (r.bytes > budget_) return false;
    std::lock_guard<std::mutex> lk(mu_);
    pending_.push_back(std::move(r));
    ++outstanding_;
    admit_locked();
    cv_.notify_all();
    return true;
  }

  // Blocks until a batch is available (true) or the scheduler is shut down
  // and has nothing left to run (false).
  bool next_batch(std::vector<Req>& batch) {
    batch.clear();
    std::unique_lock<std::mutex> lk(mu_);
    cv_.wait(lk, [&] { return !admitted_.empty() || stop_; });
    if (admitted_.empty()) return false;
    int channels = admitted_.front().D;
    const uint64_t key = admitted_.front().key;
    batch.push_back(std::move(admitted_.front()));
    admitted_.pop_front();
    for (auto it = admitted_.begin(); it != admitted_.end() && (int)batch.size() < max_sets_;) {
      if (it->key == key && channels + it->D <= max_channels_) {
        channels += it->D;
        batch.push_back(std::move(*it));
        it = admitted_.erase(it);
      } else {
        ++it;
      }
    }
    ++running_;
    return true;
  }

  // A pass has finished: its memory returns to the budget.
  void complete(const std::vector<Req>& batch) {
    std::lock_guard<std::mutex> lk(mu_);
    for (const Req& r : batch) {
      used_ -= r.bytes;
      --outstanding_;
    }
    --running_;
    admit_locked();
    cv_.notify_all();
  }

  // Removes the oldest waiting request (pending or admitted, not running)
  // for which pred holds, moving it into *out; false if there is none.
  template <typename Pred>
  bool cancel(Pred pred, Req* out) {
    std::lock_guard<std::mutex> lk(mu_);
    for (auto it = admitted_.begin(); it != admitted_.end(); ++it) {
      if (!pred(*it)) continue;
      *out = std::move(*it);
      admitted_.erase(it);
      used_ -= out->bytes;
      --outstanding_;
      admit_locked();
      cv_.notify_all();
      return true;
    }
    for (auto it = pending_.begin(); it != pending_.end(); ++it) {
      if (!pred(*it)) continue;
      *out = std::move(*it);
      pending_.erase(it);
      --outstanding_;
      admit_locked();  // a cancelled head may have been blocking the others
      cv_.notify_all();
      return true;
    }
    return false;
  }

  // Blocks until every submitted request has completed.
  void drain() {
    std::unique_lock<std::mutex> lk(mu_);
    cv_.wait(lk, [&] { return outstanding_ == 0; });
  }

  void shutdown() {
    std::lock_guard<std::mutex> lk(mu_);
    stop_ = true;
    cv_.notify_all();
  }

  int64_t used() {
    std::lock_guard<std::mutex> lk(mu_);
    return used_;
  }
  int64_t peak_used() {
    std::lock_guard<std::mutex> lk(mu_);
    return peak_;
  }

 private:
  void admit_locked() {
    while (!pending_.empty() && used_ + pending_.front().bytes <= budget_) {
      used_ += pending_.front().bytes;
      if (used_ > peak_) peak_ = used_;
      if (on_admit_) on_admit_(pending_.front());
      admitted_.push_back(std::move(pending_.front()));
      pending_.pop_front();
    }
  }

  const int64_t budget_;
  const int max_sets_, max_channels_;
  std::function<void(Req&)> on_admit_;
  std::mutex mu_;
  std::condition_variable cv_;
  std::deque<Req> pending_, admitted_;
  int64_t used_ = 0, peak_ = 0;
  int64_t outstanding_ = 0;
  int running_ = 0;
  bool stop_ = false;
};

// Runs a pass over all n requests of a batch: run(indices) -> status (0 =
// success).  If the merged pass fails with a status other than `fatal` (a
// device fault, which taints the device for every request), each request
// runs again alone, so that every request gets its own status.  Returns the
// status of each request.
template <typename Run>
std::vector<int> run_isolated(size_t n, int fatal, Run run) {
  std::vector<size_t> all(n);
  for (size_t k = 0; k < n; k++) all[k] = k;
  const int st = run(all);
  std::vector<int> out(n, st);
  if (st == 0 || n == 1 || st == fatal) return out;
  for (size_t k = 0; k < n; k++) out[k] = run(std::vector<size_t>{k});
  return out;
}

}  // namespace lv
