// Host-only check of the octree builder's thread pool (hostpool.h): every
// index of [0, n) visited exactly once for sizes around the chunk and
// single-call boundaries, an exception thrown on any participant rethrown
// on the caller (and the pool usable afterwards), calls from two threads
// serialised.  Prints "ok" and exits 0 on success.
#include <atomic>
#include <cstdio>
#include <stdexcept>
#include <thread>
#include <vector>

#include "hostpool.h"

using ccdvm::HostPool;

static bool cover(int n) {
  std::vector<std::atomic<int>> hit(n > 0 ? n : 1);
  for (auto& h : hit) h = 0;
  HostPool::get().run(n, [&](int b, int e) {
    for (int i = b; i < e; ++i) hit[i]++;
  });
  for (int i = 0; i < n; ++i)
    if (hit[i] != 1) { std::printf("n=%d: index %d visited %d times\n", n, i, (int)hit[i]); return false; }
  return true;
}

int main() {
  HostPool& pool = HostPool::get();
  const int K = HostPool::kChunk;
  for (int n : {0, 1, K - 1, K, K + 1, 2 * K, 2 * K + 1, 1000, 10007, 100003})
    if (!cover(n)) return 1;
  // an exception from a late chunk (a worker's, with several participants)
  for (int rep = 0; rep < 3; ++rep) {
    bool caught = false;
    try {
      pool.run(100 * K, [&](int b, int) {
        if (b == 97 * K) throw std::runtime_error("chunk 97");
      });
    } catch (const std::runtime_error& e) {
      caught = std::string(e.what()) == "chunk 97";
    }
    if (!caught) { std::printf("exception not rethrown (rep %d)\n", rep); return 1; }
    if (!cover(5000)) return 1;
  }
  // two callers at once
  std::atomic<long long> s1{0}, s2{0};
  std::thread t([&] {
    for (int r = 0; r < 50; ++r) pool.run(20000, [&](int b, int e) { long long s = 0; for (int i = b; i < e; ++i) s += i; s1 += s; });
  });
  for (int r = 0; r < 50; ++r) pool.run(30000, [&](int b, int e) { long long s = 0; for (int i = b; i < e; ++i) s += i; s2 += s; });
  t.join();
  if (s1 != 50LL * 20000 * 19999 / 2 || s2 != 50LL * 30000 * 29999 / 2) { std::printf("concurrent sums wrong\n"); return 1; }
  std::printf("ok %d participants\n", pool.participants());
  return 0;
}
