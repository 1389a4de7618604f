// Multi-threaded enqueue of a command-queue structure (the dispatch step of Algorithm 1,
// Sec. IV-B, where a child thread sets up and flushes the queues of each task component).
//
// Host thread t enqueues the ops of the streams s with s mod T == t, in host order.  A wait on an
// op of another stream may only be enqueued after that op's event record has been enqueued (a
// HIP event wait sees only records already issued), so before enqueueing a wait the thread spins
// until the owner of the awaited op has published it.  The host-side waits follow stream order
// and the schedule's waits, which form a DAG (host order is a topological order of it), so the
// threads cannot deadlock.  Thread 0 is the caller's thread; the others are persistent and park
// on a condition variable after a short spin when idle.  Errors in any thread abort the others'
// spins and are rethrown to the caller.
#pragma once

#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "core.hpp"

namespace psc {

// What the dispatcher does per op; the HIP runtime implements it, and a recording backend checks
// the threading on the CPU.
struct Backend {
  virtual ~Backend() = default;
  virtual void wait(int32_t op, int32_t awaited) = 0;  // stream of `op` waits on `awaited`'s event
  virtual void exec(int32_t op) = 0;                   // the op itself (kernel launch or copy)
  virtual void record(int32_t op) = 0;                 // record `op`'s event on its stream
  virtual void stream_done(int32_t stream) = 0;        // all ops of `stream` are enqueued
};

class Dispatcher {
 public:
  Dispatcher(const SchedPlan &plan, int32_t n_threads);
  ~Dispatcher();
  Dispatcher(const Dispatcher &) = delete;
  Dispatcher &operator=(const Dispatcher &) = delete;

  // Enqueues every op through `b`; returns once all threads have finished enqueueing.
  void run(Backend &b);
  int32_t threads() const { return n_threads_; }

 private:
  void work(int32_t t);
  void worker_main(int32_t t);

  const SchedPlan &plan_;
  int32_t n_threads_;
  std::vector<std::vector<int32_t>> ops_of_;  // per thread: op ids in host order
  std::vector<int32_t> streams_of_thread_;
  std::unique_ptr<std::atomic<uint64_t>[]> published_;  // per op: run generation it was issued in
  std::atomic<uint64_t> gen_{0};
  std::atomic<int32_t> finished_{0};
  std::atomic<bool> abort_{false};
  Backend *backend_ = nullptr;
  std::mutex mu_;
  std::condition_variable cv_, done_cv_;
  bool stop_ = false;
  std::string error_msg_;
  psc_status error_status_ = PSC_OK;
  std::vector<std::thread> workers_;
};

}  // namespace psc
