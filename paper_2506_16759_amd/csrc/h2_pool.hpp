// Persistent host worker pool for the planning steps (tree, block lists,
// batched layouts).  Threads are created once per process and reused, so a
// parallel loop costs a wake-up instead of thread creation and joining.
//
// parallel_for(n, f) runs f(i) for every i in [0, n) on the calling thread and
// up to 15 workers (16 participants: the host CPU share assumed for one GPU).
// A loop started from inside another one, or while a different host thread
// holds the pool, runs serially on the calling thread, so nesting is safe.
// In a child forked after the pool started (the workers are not copied into
// it) every loop runs serially.
// The first exception thrown by f is rethrown on the caller once every
// participant has stopped; the remaining indices are skipped.
#pragma once

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <exception>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

#include <unistd.h>

namespace h2 {

class HostPool {
 public:
  static HostPool& get() {
    // intentionally leaked: workers may still be parked at process exit
    static HostPool* p = new HostPool();
    return *p;
  }

  int participants() const { return static_cast<int>(workers_.size()) + 1; }

  template <typename F>
  void parallel_for(int n, int grain, F&& f) {
    if (n <= 0) return;
    grain = std::max(1, grain);
    std::unique_lock<std::mutex> busy(busy_, std::try_to_lock);
    if (in_worker() || !busy.owns_lock() || workers_.empty() || n <= grain || getpid() != pid_) {
      for (int i = 0; i < n; ++i) f(i);
      return;
    }
    std::atomic<int> next{0};
    std::atomic<bool> failed{false};
    std::exception_ptr err;
    std::mutex err_m;
    std::function<void()> body = [&] {
      for (;;) {
        const int i0 = next.fetch_add(grain);
        if (i0 >= n || failed.load(std::memory_order_relaxed)) break;
        const int i1 = std::min(n, i0 + grain);
        try {
          for (int i = i0; i < i1; ++i) f(i);
        } catch (...) {
          std::lock_guard<std::mutex> g(err_m);
          if (!err) err = std::current_exception();
          failed = true;
        }
      }
    };
    const int want = std::min(static_cast<int>(workers_.size()), (n + grain - 1) / grain - 1);
    {
      std::lock_guard<std::mutex> g(m_);
      job_ = &body;
      pending_ = want;
      running_ = want;
      ++gen_;
    }
    cv_.notify_all();
    in_worker() = true;
    body();
    in_worker() = false;
    {
      std::unique_lock<std::mutex> g(m_);
      done_.wait(g, [&] { return running_ == 0; });
      job_ = nullptr;
    }
    if (err) std::rethrow_exception(err);
  }

 private:
  HostPool() : pid_(getpid()) {
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const int nw = static_cast<int>(std::min(hw, 16u)) - 1;
    for (int w = 0; w < nw; ++w) workers_.emplace_back([this] { loop(); });
    for (auto& t : workers_) t.detach();
  }

  static bool& in_worker() {
    thread_local bool flag = false;
    return flag;
  }

  void loop() {
    in_worker() = true;
    uint64_t seen = 0;
    for (;;) {
      std::function<void()>* job;
      {
        std::unique_lock<std::mutex> g(m_);
        cv_.wait(g, [&] { return gen_ != seen && pending_ > 0; });
        seen = gen_;
        --pending_;
        job = job_;
      }
      (*job)();
      {
        std::lock_guard<std::mutex> g(m_);
        if (--running_ == 0) done_.notify_one();
      }
    }
  }

  const pid_t pid_;
  std::vector<std::thread> workers_;
  std::mutex busy_, m_;
  std::condition_variable cv_, done_;
  std::function<void()>* job_ = nullptr;
  uint64_t gen_ = 0;
  int pending_ = 0, running_ = 0;
};

template <typename F>
inline void parallel_for(int n, int grain, F&& f) {
  HostPool::get().parallel_for(n, grain, std::forward<F>(f));
}

}  // namespace h2
