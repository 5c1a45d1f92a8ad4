// Admission policy of the serving runtime: which pending requests go into
// the next batch of a free device slot.  Plain C++ (no HIP), so the policy
// is unit-tested on the CPU.
//
// A request is admitted in arrival order while the batch stays within the
// slot's capacities: graphs, vertices, adjacency entries, and root slots.
// Root slots are the memory estimate: a graph needs at most
// sum over its vertices of C(deg, 2) initial triplets (stage one never
// produces more), each held in device memory until the depth-first kernel
// consumes it; the depth-first stacks are a fixed per-slot workspace.  A
// request that could never fit an empty slot is rejected.
#pragma once

#include <cstdint>
#include <deque>
#include <vector>

namespace ccserve {

struct Capacity {
  int64_t graphs = 256;
  int64_t vertices = 256 * 256;  // graphs times the largest graph
  int64_t entries = 1 << 21;  // adjacency entries (2m)
  int64_t roots = 1 << 22;
};

struct Cost {
  int64_t vertices = 0;
  int64_t entries = 0;
  int64_t roots = 0;
};

// Memory estimate of one graph from its CSR (degrees only).
inline Cost cost_of(int32_t n, const int32_t *row_ptr) {
  Cost c;
  c.vertices = n;
  c.entries = n > 0 ? row_ptr[n] - row_ptr[0] : 0;
  for (int32_t v = 0; v < n; ++v) {
    const int64_t d = row_ptr[v + 1] - row_ptr[v];
    c.roots += d * (d - 1) / 2;
  }
  return c;
}

inline bool fits_empty(const Cost &c, const Capacity &cap) {
  return c.vertices <= cap.vertices && c.entries <= cap.entries && c.roots <= cap.roots &&
         cap.graphs >= 1;
}

// Takes requests from the front of `pending` (ids with their costs) while
// they fit; stops at the first that does not (arrival order is kept).
// Returns the admitted ids.
template <typename Id>
std::vector<Id> admit(std::deque<std::pair<Id, Cost>> &pending, const Capacity &cap) {
  std::vector<Id> out;
  Cost used;
  while (!pending.empty() && (int64_t)out.size() < cap.graphs) {
    const Cost &c = pending.front().second;
    if (used.vertices + c.vertices > cap.vertices || used.entries + c.entries > cap.entries ||
        used.roots + c.roots > cap.roots)
      break;
    used.vertices += c.vertices;
    used.entries += c.entries;
    used.roots += c.roots;
    out.push_back(pending.front().first);
    pending.pop_front();
  }
  return out;
}

}  // namespace ccserve
