// Multi-threaded enqueue; see dispatch.hpp.
#include "dispatch.hpp"

#include <chrono>

#if defined(__x86_64__)
#include <immintrin.h>
#define PSC_PAUSE() _mm_pause()
#else
#define PSC_PAUSE() ((void)0)
#endif

namespace psc {

namespace {
using Clock = std::chrono::steady_clock;
constexpr auto kIdleSpin = std::chrono::milliseconds(20);  // spin before parking when idle
}  // namespace

Dispatcher::Dispatcher(const SchedPlan &plan, int32_t n_threads)
    : plan_(plan), n_threads_(std::max<int32_t>(1, std::min(n_threads, plan.total_streams))) {
  ops_of_.assign(n_threads_, {});
  for (size_t o = 0; o < plan_.ops.size(); ++o)
    ops_of_[plan_.ops[o].stream % n_threads_].push_back(static_cast<int32_t>(o));
  published_.reset(new std::atomic<uint64_t>[plan_.ops.size() ? plan_.ops.size() : 1]);
  for (size_t o = 0; o < plan_.ops.size(); ++o) published_[o].store(0, std::memory_order_relaxed);
  for (int32_t t = 1; t < n_threads_; ++t) workers_.emplace_back([this, t] { worker_main(t); });
}

Dispatcher::~Dispatcher() {
  {
    std::lock_guard<std::mutex> lk(mu_);
    stop_ = true;
  }
  cv_.notify_all();
  for (auto &w : workers_) w.join();
}

void Dispatcher::work(int32_t t) {
  const uint64_t g = gen_.load(std::memory_order_acquire);
  try {
    for (int32_t o : ops_of_[t]) {
      const Op &op = plan_.ops[o];
      for (int32_t w : op.waits) {
        // the awaited op's record must already be enqueued by its owner
        while (published_[w].load(std::memory_order_acquire) < g) {
          if (abort_.load(std::memory_order_relaxed)) return;
          PSC_PAUSE();
        }
        backend_->wait(o, w);
      }
      backend_->exec(o);
      if (op.recorded) backend_->record(o);
      published_[o].store(g, std::memory_order_release);
    }
    for (int32_t s = t; s < plan_.total_streams; s += n_threads_) backend_->stream_done(s);
  } catch (const Error &e) {
    std::lock_guard<std::mutex> lk(mu_);
    if (error_status_ == PSC_OK) {
      error_status_ = e.status;
      error_msg_ = e.msg;
    }
    abort_.store(true);
  } catch (const std::exception &e) {
    std::lock_guard<std::mutex> lk(mu_);
    if (error_status_ == PSC_OK) {
      error_status_ = PSC_ERR_ARG;
      error_msg_ = e.what();
    }
    abort_.store(true);
  }
}

void Dispatcher::worker_main(int32_t t) {
  uint64_t seen = 0;
  for (;;) {
    // spin briefly for the next run, then park
    const auto t0 = Clock::now();
    while (gen_.load(std::memory_order_acquire) == seen) {
      if (Clock::now() - t0 > kIdleSpin) {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [&] { return stop_ || gen_.load(std::memory_order_acquire) != seen; });
        if (stop_) return;
        break;
      }
      PSC_PAUSE();
    }
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (stop_) return;
    }
    seen = gen_.load(std::memory_order_acquire);
    work(t);
    if (finished_.fetch_add(1, std::memory_order_acq_rel) + 1 == n_threads_ - 1) {
      std::lock_guard<std::mutex> lk(mu_);
      done_cv_.notify_all();
    }
  }
}

void Dispatcher::run(Backend &b) {
  backend_ = &b;
  abort_.store(false);
  error_status_ = PSC_OK;
  error_msg_.clear();
  finished_.store(0, std::memory_order_relaxed);
  {
    std::lock_guard<std::mutex> lk(mu_);
    gen_.fetch_add(1, std::memory_order_acq_rel);
  }
  cv_.notify_all();
  work(0);
  // wait for the other threads: spin, then block
  const auto t0 = Clock::now();
  while (finished_.load(std::memory_order_acquire) < n_threads_ - 1) {
    if (Clock::now() - t0 > kIdleSpin) {
      std::unique_lock<std::mutex> lk(mu_);
      done_cv_.wait(lk, [&] { return finished_.load(std::memory_order_acquire) >= n_threads_ - 1; });
      break;
    }
    PSC_PAUSE();
  }
  backend_ = nullptr;
  if (error_status_ != PSC_OK) fail(error_status_, error_msg_);
}

}  // namespace psc
