// CPU checks of the serving admission policy (cc_serve_policy.h): cost
// estimate, capacity limits, arrival order, and a simulated request loop
// with a fake executor in which every request is answered exactly once.
// Prints "ok" and exits 0 on success; prints the failed check and exits 1.
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <vector>

#include "cc_serve_policy.h"

#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) {                                                    \
      std::printf("FAILED %s:%d: %s\n", __FILE__, __LINE__, #c);   \
      std::exit(1);                                                \
    }                                                              \
  } while (0)

using ccserve::Capacity;
using ccserve::Cost;

static Cost cost(int64_t v, int64_t e, int64_t r) {
  Cost c;
  c.vertices = v;
  c.entries = e;
  c.roots = r;
  return c;
}

int main() {
  // cost_of on the star K_{1,4} plus an isolated vertex: centre degree 4
  // gives C(4,2) = 6 root slots, the leaves none.
  {
    const int32_t rp[] = {0, 4, 5, 6, 7, 8, 8};
    const Cost c = ccserve::cost_of(6, rp);
    CHECK(c.vertices == 6 && c.entries == 8 && c.roots == 6);
    const int32_t rp0[] = {0};
    const Cost z = ccserve::cost_of(0, rp0);
    CHECK(z.vertices == 0 && z.entries == 0 && z.roots == 0);
  }
  // capacity limits, each on its own
  {
    Capacity cap;
    cap.graphs = 3;
    cap.vertices = 100;
    cap.entries = 1000;
    cap.roots = 50;
    std::deque<std::pair<int, Cost>> q;
    for (int i = 0; i < 5; ++i) q.emplace_back(i, cost(10, 10, 1));
    std::vector<int> a = ccserve::admit(q, cap);  // graph count binds
    CHECK(a.size() == 3 && a[0] == 0 && a[1] == 1 && a[2] == 2 && q.size() == 2);
    q.clear();
    q.emplace_back(0, cost(60, 1, 1));
    q.emplace_back(1, cost(50, 1, 1));  // vertices: 110 > 100
    q.emplace_back(2, cost(1, 1, 1));   // would fit, but order is kept
    a = ccserve::admit(q, cap);
    CHECK(a.size() == 1 && a[0] == 0 && q.front().first == 1);
    q.clear();
    q.emplace_back(0, cost(1, 1, 30));
    q.emplace_back(1, cost(1, 1, 20));  // roots: exactly 50 fits
    q.emplace_back(2, cost(1, 1, 1));
    a = ccserve::admit(q, cap);
    CHECK(a.size() == 2 && q.size() == 1);
    q.clear();
    q.emplace_back(0, cost(1, 600, 1));
    q.emplace_back(1, cost(1, 401, 1));  // entries: 1001 > 1000
    a = ccserve::admit(q, cap);
    CHECK(a.size() == 1);
    CHECK(ccserve::fits_empty(cost(100, 1000, 50), cap));
    CHECK(!ccserve::fits_empty(cost(101, 0, 0), cap));
    CHECK(!ccserve::fits_empty(cost(0, 1001, 0), cap));
    CHECK(!ccserve::fits_empty(cost(0, 0, 51), cap));
    std::deque<std::pair<int, Cost>> empty;
    CHECK(ccserve::admit(empty, cap).empty());
  }
  // simulated loop: 3 slots, random arrivals and batch durations; every
  // request is answered once, admissions follow arrival order, and every
  // batch respects the capacities
  {
    std::mt19937_64 rng(14104876);
    Capacity cap;
    cap.graphs = 8;
    cap.vertices = 400;
    cap.entries = 4000;
    cap.roots = 3000;
    const int n_req = 5000;
    std::deque<std::pair<int, Cost>> pending;
    std::map<int, int> answered;
    struct Slot {
      bool busy = false;
      int64_t t_end = 0;
      std::vector<int> reqs;
    };
    std::vector<Slot> slots(3);
    int next = 0, last_admitted = -1;
    int64_t t = 0;
    while ((int)answered.size() < n_req) {
      ++t;
      if (next < n_req && rng() % 3 == 0) {
        const int64_t v = 3 + (int64_t)(rng() % 126);
        const int64_t e = v * (2 + (int64_t)(rng() % 6));
        const int64_t r = (int64_t)(rng() % 3001);
        pending.emplace_back(next++, cost(v, e, r));
      }
      for (Slot &s : slots) {
        if (s.busy && s.t_end <= t) {
          for (int id : s.reqs) answered[id]++;
          s.reqs.clear();
          s.busy = false;
        }
        if (!s.busy && !pending.empty()) {
          Cost sum;
          std::map<int, Cost> costs;
          for (auto &p : pending) costs[p.first] = p.second;
          s.reqs = ccserve::admit(pending, cap);
          CHECK(!s.reqs.empty());  // every generated request fits an empty slot
          CHECK((int64_t)s.reqs.size() <= cap.graphs);
          for (int id : s.reqs) {
            CHECK(id == last_admitted + 1);
            last_admitted = id;
            sum.vertices += costs[id].vertices;
            sum.entries += costs[id].entries;
            sum.roots += costs[id].roots;
          }
          CHECK(sum.vertices <= cap.vertices && sum.entries <= cap.entries &&
                sum.roots <= cap.roots);
          s.busy = true;
          s.t_end = t + 1 + (int64_t)(rng() % 20);
        }
      }
      CHECK(t < 10000000);
    }
    CHECK((int)answered.size() == n_req);
    for (auto &kv : answered) CHECK(kv.second == 1);
  }
  std::printf("ok\n");
  return 0;
}
