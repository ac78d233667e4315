// A small persistent pool of host threads for the library's host-side work
// (op compilation, run grouping): tasks 0..n-1 of one job run on the workers
// and the calling thread, and run() returns when all are done.  Jobs from
// different callers are serialised; a task that itself asks for parallel work
// gets it run serially on its own thread.
#pragma once

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstddef>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

namespace sparsesim {

class HostPool {
 public:
  static constexpr unsigned kMaxThreads = 16;  // including the caller

  static HostPool& get() {
    static HostPool pool;
    return pool;
  }

  unsigned threads() const { return (unsigned)workers_.size() + 1; }
  // Parallel work asked for by the calling thread runs serially on it from
  // now on (for the library's other worker threads, so that they never wait
  // for this pool's jobs).
  static void run_serially_here() { in_task() = true; }

  // fn(i) for i in [0, n); blocks until every task has finished and every
  // worker has left the job.
  void run(size_t n, const std::function<void(size_t)>& fn) {
    if (n == 0) return;
    if (n == 1 || workers_.empty() || in_task()) {
      for (size_t i = 0; i < n; ++i) fn(i);
      return;
    }
    std::lock_guard<std::mutex> job_lock(job_mu_);
    Job job;
    job.fn = &fn;
    job.n = n;
    job.left.store(n);
    {
      std::lock_guard<std::mutex> lk(mu_);
      job_ = &job;
      ++generation_;
    }
    cv_.notify_all();
    work(job);
    std::unique_lock<std::mutex> lk(mu_);
    done_cv_.wait(lk, [&] { return job.left.load() == 0; });
    job_ = nullptr;   // no worker joins from here on
    done_cv_.wait(lk, [&] { return job.active == 0; });
  }

  ~HostPool() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
      ++generation_;
    }
    cv_.notify_all();
    for (auto& t : workers_) t.join();
  }

 private:
  struct Job {
    const std::function<void(size_t)>* fn = nullptr;
    size_t n = 0;
    std::atomic<size_t> next{0}, left{0};
    int active = 0;   // workers inside work(), guarded by mu_
  };

  HostPool() {
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const unsigned n = std::min(kMaxThreads, hw) - 1;
    for (unsigned i = 0; i < n; ++i) workers_.emplace_back([this] { loop(); });
  }

  static bool& in_task() {
    static thread_local bool flag = false;
    return flag;
  }

  // Take tasks of the job until none are left.
  void work(Job& job) {
    in_task() = true;
    for (;;) {
      const size_t i = job.next.fetch_add(1);
      if (i >= job.n) break;
      (*job.fn)(i);
      if (job.left.fetch_sub(1) == 1) {
        std::lock_guard<std::mutex> lk(mu_);
        done_cv_.notify_all();
      }
    }
    in_task() = false;
  }

  void loop() {
    size_t seen = 0;
    for (;;) {
      Job* job = nullptr;
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [&] { return stop_ || generation_ != seen; });
        if (stop_) return;
        seen = generation_;
        job = job_;
        if (!job) continue;
        ++job->active;
      }
      work(*job);
      std::lock_guard<std::mutex> lk(mu_);
      --job->active;
      done_cv_.notify_all();
    }
  }

  std::vector<std::thread> workers_;
  std::mutex job_mu_, mu_;
  std::condition_variable cv_, done_cv_;
  Job* job_ = nullptr;
  size_t generation_ = 0;
  bool stop_ = false;
};

// f(begin, end, part) over [0, n) cut into at most threads() parts of at
// least min_part items each (one part, on the caller, when n is small).
template <class F>
void parallel_parts(size_t n, size_t min_part, F&& f) {
  HostPool& pool = HostPool::get();
  const size_t parts = std::min<size_t>(pool.threads(), n / std::max<size_t>(min_part, 1));
  if (parts <= 1) {
    f(size_t(0), n, size_t(0));
    return;
  }
  pool.run(parts, [&](size_t p) { f(n * p / parts, n * (p + 1) / parts, p); });
}

}  // namespace sparsesim
