// The serving loop's admission (p1e_admission.h, the code p1e_server_step uses) driven by a
// fake executor on the CPU: requests with Poisson arrivals (seeded exponential gaps) and
// log-uniform sizes, each holding pool bytes and a slot for a number of engine steps
// proportional to its size. Every step retires the finished requests, then admits waiting
// ones in arrival order. Checked at every step: allocated blocks disjoint and inside the pool,
// free blocks coalesced and summing with the allocated ones to the pool, one request per slot,
// admission in arrival order, a waiting head of line that really does not fit, and at the end
// every request served or (larger than the pool) refused. With one slot and an ample pool the
// loop is a FIFO single-server queue: its finish times, and so its latency percentiles, must
// equal those of the queue's recursion start = max(arrival, previous finish).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <deque>
#include <random>
#include <vector>

#include "p1e_admission.h"

using p1e::Admission;
using p1e::Admit;

static int g_fail = 0;
#define CHECK(c, ...)                                                             \
  do {                                                                            \
    if (!(c)) {                                                                   \
      std::fprintf(stderr, "check failed (line %d): %s: ", __LINE__, #c);        \
      std::fprintf(stderr, __VA_ARGS__);                                          \
      std::fprintf(stderr, "\n");                                                 \
      if (++g_fail > 20) return {};                                               \
    }                                                                             \
  } while (0)

struct Req {
  int64_t arrive;  // step of arrival
  uint64_t bytes;
  int64_t steps;   // engine steps it needs once admitted
  int64_t admit = -1, finish = -1;
  int slot = -1;
  uint64_t off = 0;
  bool refused = false;
};

static double pct(std::vector<double> x, double q) {
  std::sort(x.begin(), x.end());
  const double pos = q / 100.0 * (x.size() - 1);
  const size_t i = (size_t)pos;
  const double f = pos - i;
  return i + 1 < x.size() ? x[i] * (1 - f) + x[i + 1] * f : x[i];
}

struct Result {
  std::vector<Req> reqs;
  int64_t steps = 0;
};

static Result run(int nreq, int slots, uint64_t pool, double rate, uint64_t seed) {
  std::mt19937_64 rng(seed);
  std::exponential_distribution<double> gap(rate);
  std::uniform_real_distribution<double> U(std::log(1e4), std::log(2e6));
  Result R;
  std::vector<Req> &q = R.reqs;
  double t = 0.0;
  for (int i = 0; i < nreq; ++i) {
    t += gap(rng);
    const double size = std::exp(U(rng));
    Req r;
    r.arrive = (int64_t)std::ceil(t);
    r.bytes = (uint64_t)(size * 100.0);
    r.steps = 1 + (int64_t)(size / 2e4);
    q.push_back(r);
  }
  if (nreq > 3) q[nreq / 2].bytes = pool + 1;  // one request that can never fit
  Admission adm;
  adm.reset(slots, pool);
  std::vector<int> active;  // request indices in slots
  size_t next = 0;          // first request not yet admitted or refused (arrival order)
  int64_t step = 0;
  while (next < q.size() || !active.empty()) {
    // 1. retire
    for (size_t a = 0; a < active.size();) {
      Req &r = q[active[a]];
      if (step - r.admit >= r.steps) {
        r.finish = step;
        adm.retire(r.slot, r.off, r.bytes);
        active[a] = active.back();
        active.pop_back();
      } else {
        ++a;
      }
    }
    // 2. admit in arrival order
    while (next < q.size() && q[next].arrive <= step) {
      Req &r = q[next];
      int slot;
      uint64_t off;
      const Admit res = adm.try_admit((int64_t)next, r.bytes, slot, off);
      if (res == Admit::kNever) {
        r.refused = true;
        CHECK(r.bytes > pool, "refused a request of %llu bytes", (unsigned long long)r.bytes);
        ++next;
        continue;
      }
      if (res == Admit::kWait) {  // the head of line really does not fit
        uint64_t big = 0;
        for (auto &b : adm.pool.free_blocks()) big = std::max(big, b.second);
        CHECK((int)active.size() == slots || big < r.bytes, "head waits though it fits");
        break;
      }
      r.admit = step;
      r.slot = slot;
      r.off = off;
      active.push_back((int)next);
      ++next;
    }
    // invariants
    std::vector<std::pair<uint64_t, uint64_t>> blk;
    uint64_t used = 0;
    std::vector<int> seen(slots, 0);
    for (int a : active) {
      blk.push_back({q[a].off, q[a].bytes});
      used += q[a].bytes;
      CHECK(q[a].slot >= 0 && q[a].slot < slots && adm.owner[q[a].slot] == a, "slot table");
      seen[q[a].slot] += 1;
    }
    for (int s2 = 0; s2 < slots; ++s2) CHECK(seen[s2] <= 1, "slot %d shared", s2);
    std::sort(blk.begin(), blk.end());
    for (size_t i = 0; i < blk.size(); ++i) {
      CHECK(blk[i].first + blk[i].second <= pool, "block past the pool");
      if (i) CHECK(blk[i - 1].first + blk[i - 1].second <= blk[i].first, "blocks overlap");
    }
    uint64_t fr = 0, prev_end = UINT64_MAX;
    for (auto &b : adm.pool.free_blocks()) {
      CHECK(b.first != prev_end, "free blocks not coalesced");
      prev_end = b.first + b.second;
      fr += b.second;
    }
    CHECK(fr + used == pool, "bytes lost: free %llu used %llu", (unsigned long long)fr,
          (unsigned long long)used);
    ++step;
    CHECK(step < 100000000, "no progress");
  }
  // arrival order of admission, all served
  int64_t last = -1;
  for (auto &r : q) {
    if (r.refused) continue;
    CHECK(r.admit >= r.arrive && r.admit >= last && r.finish == r.admit + r.steps, "order/timing");
    last = r.admit;
  }
  R.steps = step;
  return R;
}

int main() {
  // mixed load: 8 slots, a pool for about a dozen requests at once
  Result a = run(2000, 8, (uint64_t)(12 * 3e5 * 100), 1.0 / 20.0, 7);
  int refused = 0;
  std::vector<double> lat;
  for (auto &r : a.reqs) {
    if (r.refused) ++refused;
    else lat.push_back((double)(r.finish - r.arrive));
  }
  std::printf("admission: %zu requests, %d refused, %lld steps, latency p50 %.1f p99 %.1f steps\n",
              a.reqs.size(), refused, (long long)a.steps, pct(lat, 50), pct(lat, 99));
  if (refused != 1) { std::fprintf(stderr, "expected one refusal\n"); ++g_fail; }
  // one slot, ample pool: the FIFO single-server queue
  Result b = run(1000, 1, (uint64_t)1 << 50, 1.0 / 40.0, 11);
  std::vector<double> lb, lr;
  int64_t fin = 0;
  for (auto &r : b.reqs) {
    if (r.refused) continue;
    const int64_t start = std::max(r.arrive, fin);
    fin = start + r.steps;
    if (r.finish != fin) { ++g_fail; std::fprintf(stderr, "finish %lld vs recursion %lld\n", (long long)r.finish, (long long)fin); break; }
    lb.push_back((double)(r.finish - r.arrive));
    lr.push_back((double)(fin - r.arrive));
  }
  std::printf("single slot: p50 %.1f p99 %.1f steps (recursion p50 %.1f p99 %.1f)\n", pct(lb, 50),
              pct(lb, 99), pct(lr, 50), pct(lr, 99));
  if (pct(lb, 50) != pct(lr, 50) || pct(lb, 99) != pct(lr, 99)) ++g_fail;
  std::printf("%d failed checks\n", g_fail);
  return g_fail ? 1 : 0;
}
