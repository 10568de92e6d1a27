// Host-only self-test of the serving engine's scheduling logic (wave_sched.h):
// first-fit pool allocation with coalescing, admission with skip-ahead, nearest-
// rank percentiles, and a simulated executor that completes admitted requests in
// simulated time, checking budget, overlap, progress and ordering invariants.
// Built with the host compiler by tests/test_sched_host.py; exits non-zero on failure.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>
#include <vector>

#include "wave_sched.h"

using namespace wave::sched;

#define CHECK(c)                                                         \
  do {                                                                   \
    if (!(c)) {                                                          \
      std::fprintf(stderr, "FAILED %s at line %d\n", #c, __LINE__);     \
      std::exit(1);                                                      \
    }                                                                    \
  } while (0)

static void test_pool() {
  PoolAlloc p(1000 * kGranule);
  size_t a, b, c, d;
  CHECK(p.alloc(100 * kGranule, &a) && a == 0);
  CHECK(p.alloc(200 * kGranule - 5, &b) && b == 100 * kGranule);  // rounded up
  CHECK(p.alloc(300 * kGranule, &c) && c == 300 * kGranule);
  CHECK(!p.alloc(401 * kGranule, &d));
  CHECK(p.alloc(400 * kGranule, &d) && d == 600 * kGranule);
  CHECK(p.free_bytes() == 0);
  p.release(b, 200 * kGranule - 5);  // hole of 200 in the middle
  CHECK(p.free_bytes() == 200 * kGranule && p.blocks() == 1);
  CHECK(!p.alloc(201 * kGranule, &d));
  p.release(a, 100 * kGranule);      // coalesces with the hole
  CHECK(p.blocks() == 1 && p.largest_free() == 300 * kGranule);
  CHECK(p.alloc(250 * kGranule, &d) && d == 0);  // first fit
  p.release(0, 250 * kGranule);
  p.release(c, 300 * kGranule);
  p.release(600 * kGranule, 400 * kGranule);
  CHECK(p.blocks() == 1 && p.largest_free() == 1000 * kGranule);
}

static void test_admit() {
  PoolAlloc p(1000 * kGranule);
  std::vector<size_t> q = {600 * kGranule, 500 * kGranule, 300 * kGranule, 200 * kGranule};
  auto adm = admit(q, p, 8);
  // the 500 does not fit after the 600; the 300 overtakes it; then 100 are left
  CHECK(adm.size() == 2 && adm[0].pos == 0 && adm[1].pos == 2);
  CHECK(adm[0].off == 0 && adm[1].off == 600 * kGranule);
  PoolAlloc p2(1000 * kGranule);
  auto adm2 = admit(q, p2, 1);  // one free slot: only the head
  CHECK(adm2.size() == 1 && adm2[0].pos == 0);
  PoolAlloc p3(1000 * kGranule);
  CHECK(admit({}, p3, 4).empty());
}

static void test_percentile() {
  std::vector<double> v;
  for (int i = 100; i >= 1; --i) v.push_back(i);
  CHECK(percentile(v, 0.50) == 50.0);
  CHECK(percentile(v, 0.99) == 99.0);
  CHECK(percentile(v, 1.00) == 100.0);
  CHECK(percentile({7.0}, 0.99) == 7.0);
  CHECK(percentile({}, 0.5) == 0.0);
  CHECK(percentile({3.0, 1.0, 2.0}, 0.5) == 2.0);
}

// Simulated executor: requests (arrival, bytes, service time); admitted requests
// run concurrently and finish after their service time.
static void test_simulation(unsigned seed) {
  std::mt19937_64 rng(seed);
  const size_t budget = 4096 * kGranule;
  const int slots = 6;
  struct Req { double arrive, service; size_t bytes; double admit = -1, done = -1; size_t off = 0; };
  std::vector<Req> reqs;
  double t = 0;
  std::uniform_real_distribution<double> U(0, 1);
  for (int i = 0; i < 300; ++i) {
    t += -std::log(1 - U(rng)) * 0.5;
    reqs.push_back({t, 0.5 + 3 * U(rng), (size_t)(64 + U(rng) * 2000) * kGranule});
  }
  PoolAlloc pool(budget);
  std::vector<int> queue, running;
  size_t next = 0;
  double now = 0;
  while (next < reqs.size() || !queue.empty() || !running.empty()) {
    // next event: an arrival or a completion
    double t_arr = next < reqs.size() ? reqs[next].arrive : 1e300;
    double t_fin = 1e300;
    int fin = -1;
    for (int r : running)
      if (reqs[r].admit + reqs[r].service < t_fin) {
        t_fin = reqs[r].admit + reqs[r].service;
        fin = r;
      }
    CHECK(t_arr < 1e300 || fin >= 0);
    if (t_arr <= t_fin) {
      now = t_arr;
      queue.push_back((int)next++);
    } else {
      now = t_fin;
      reqs[fin].done = now;
      pool.release(reqs[fin].off, reqs[fin].bytes);
      running.erase(std::find(running.begin(), running.end(), fin));
    }
    std::vector<size_t> qb;
    for (int r : queue) qb.push_back(reqs[r].bytes);
    auto adm = admit(qb, pool, slots - (int)running.size());
    std::set<size_t> admitted;
    for (auto& a : adm) {
      Req& r = reqs[queue[a.pos]];
      r.admit = now;
      r.off = a.off;
      running.push_back(queue[a.pos]);
      admitted.insert(a.pos);
    }
    std::vector<int> rest;
    for (size_t i = 0; i < queue.size(); ++i)
      if (!admitted.count(i)) rest.push_back(queue[i]);
    queue.swap(rest);
    // invariants: within budget and slots, live allocations disjoint
    size_t used = 0;
    std::vector<std::pair<size_t, size_t>> iv;
    for (int r : running) {
      used += round_up(reqs[r].bytes);
      iv.push_back({reqs[r].off, reqs[r].off + round_up(reqs[r].bytes)});
    }
    CHECK(used <= budget && (int)running.size() <= slots);
    std::sort(iv.begin(), iv.end());
    for (size_t i = 1; i < iv.size(); ++i) CHECK(iv[i - 1].second <= iv[i].first);
    CHECK(used + pool.free_bytes() == budget);
    // a request left waiting could not have been placed with a free slot
    if (!queue.empty() && (int)running.size() < slots)
      for (int r : queue) CHECK(pool.largest_free() < round_up(reqs[r].bytes));
  }
  std::vector<double> lat;
  for (auto& r : reqs) {
    CHECK(r.admit >= r.arrive && r.done >= r.admit + r.service - 1e-9);
    lat.push_back(r.done - r.arrive);
  }
  CHECK(percentile(lat, 0.5) <= percentile(lat, 0.99));
  CHECK(pool.blocks() == 1 && pool.free_bytes() == budget);
}

int main() {
  test_pool();
  test_admit();
  test_percentile();
  for (unsigned s = 1; s <= 20; ++s) test_simulation(s);
  std::printf("sched selftest OK\n");
  return 0;
}
