// A small pool of host threads for the per-leaf loops of the octree
// builder (one pool per process, created on first use and never destroyed:
// its threads end with the process).  run(n, fn) calls fn(begin, end) over
// chunks of [0, n) of kChunk items, chunk c on participant c % P (the
// calling thread is participant 0), and returns when every participant is
// done.  Every worker takes part in every call, so a call cannot start
// before all workers have finished the previous one; calls from several
// threads are serialised.  A waiting thread spins for a few tens of
// microseconds before it sleeps (a mesh build makes a few dozen calls in a
// row).  An exception thrown by fn on any participant
// (the first one caught) is rethrown by run on the calling thread once
// every participant is done.
#pragma once

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <exception>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

namespace ccdvm {

class HostPool {
 public:
  static constexpr int kChunk = 64;

  static HostPool& get() {
    static HostPool* p = new HostPool();
    return *p;
  }

  int participants() const { return nw_ + 1; }

  void run(int n, const std::function<void(int, int)>& fn) {
    if (n <= 0) return;
    if (nw_ == 0 || n <= 2 * kChunk) { fn(0, n); return; }
    std::lock_guard<std::mutex> serial(call_);
    {
      std::lock_guard<std::mutex> lk(m_);
      fn_ = &fn; n_ = n;
      error_ = nullptr;
      pending_.store(nw_, std::memory_order_relaxed);
      gen_.store(gen_.load(std::memory_order_relaxed) + 1, std::memory_order_release);
    }
    cv_.notify_all();
    slice(0, fn, n);
    spin_until([&] { return pending_.load(std::memory_order_acquire) == 0; });
    if (pending_.load(std::memory_order_acquire) != 0) {
      std::unique_lock<std::mutex> lk(m_);
      fin_.wait(lk, [&] { return pending_.load(std::memory_order_acquire) == 0; });
    }
    if (error_) {
      std::exception_ptr e = error_;
      error_ = nullptr;
      std::rethrow_exception(e);
    }
  }

 private:
  static constexpr std::chrono::microseconds kSpin{50};

  template <class Pred>
  static void spin_until(Pred&& done) {
    const auto t0 = std::chrono::steady_clock::now();
    for (int k = 1; !done(); ++k) {
      __builtin_ia32_pause();
      if ((k & 63) == 0 && std::chrono::steady_clock::now() - t0 > kSpin) return;
    }
  }

  HostPool() {
    // at most 12 participants: with the 16 host CPUs one GPU gets, the rest
    // is left to the thread that drives the device, the concurrent mesh
    // build's caller and the HIP runtime (12 measured faster than 8 or 16,
    // and leaves room for the spinning)
    const unsigned hw = std::thread::hardware_concurrency();
    const int want = (int)std::max(1u, std::min(hw, 12u)) - 1;
    // the workers that could be started (a thread that cannot start leaves
    // the pool smaller, not broken); they first read nw_ in a call
    for (int t = 1; t <= want; ++t) {
      try {
        std::thread([this, t] { loop(t); }).detach();
      } catch (...) {
        break;
      }
      nw_ = t;
    }
  }

  // the participant's chunks; it stops at the first exception and keeps it
  void slice(int id, const std::function<void(int, int)>& f, int n) {
    const int P = nw_ + 1;
    try {
      for (long long c = id; c * kChunk < n; c += P)
        f((int)(c * kChunk), (int)std::min<long long>(n, (c + 1) * kChunk));
    } catch (...) {
      std::lock_guard<std::mutex> lk(m_);
      if (!error_) error_ = std::current_exception();
    }
  }

  // fn_ and n_ are written before the release store of gen_ and read after
  // the acquire load that sees it; a call cannot start before every worker
  // has finished the previous one, so no generation is skipped
  void loop(int id) {
    unsigned long long seen = 0;
    for (;;) {
      spin_until([&] { return gen_.load(std::memory_order_acquire) != seen; });
      if (gen_.load(std::memory_order_acquire) == seen) {
        std::unique_lock<std::mutex> lk(m_);
        cv_.wait(lk, [&] { return gen_.load(std::memory_order_acquire) != seen; });
      }
      seen = gen_.load(std::memory_order_acquire);
      slice(id, *fn_, n_);
      if (pending_.fetch_sub(1, std::memory_order_acq_rel) == 1) {
        std::lock_guard<std::mutex> lk(m_);
        fin_.notify_all();
      }
    }
  }

  int nw_ = 0;
  std::mutex m_, call_;
  std::condition_variable cv_, fin_;
  const std::function<void(int, int)>* fn_ = nullptr;
  int n_ = 0;
  std::atomic<int> pending_{0};
  std::exception_ptr error_;
  std::atomic<unsigned long long> gen_{0};
};

}  // namespace ccdvm
