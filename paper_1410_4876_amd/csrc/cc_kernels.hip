// HIP kernels for chordless-cycle enumeration on gfx950 (MI355X).
//
// Vertices are renumbered by their degree label (Section 2), so "label
// greater than the label of v2" is an integer comparison and every vertex
// set is a W-word bitset (W = 1, 2, 4, 8 or 16 for n <= 64, 128, 256, 512,
// 1024).  An open chordless path p = <v1, ..., vt> is carried as
// (X, S, v1, vt) where
//   X = N(v2) U ... U N(v(t-1)) U {w : w <= v2}   (the exclusion set)
//   S = {v1, ..., vt}                               (enumerate mode only)
// For the next vertex, Algorithm 3's tests (v not on p, label above v2, no
// neighbour among v2..v(t-1)) are exactly "v in N(vt) \ X": every vertex of
// p already lies in X (v1 and v(i-1) are neighbours of internal vertices, v2
// is below-or-equal itself).  Of those candidates, the ones adjacent to v1
// close a chordless cycle <p, v>; the others extend p, with
// X' = X | N(vt), S' = S | {v} (Algorithm 1, the three cases of its loop).
// The path-extension property of Section 2 guarantees there is no other
// case.
#include <atomic>

#include "cc_internal.h"

namespace {

// ------------------------------------------------------------- bitsets
template <int W>
struct Bits {
  unsigned long long w[W];
};

template <int W>
__device__ __forceinline__ Bits<W> row(const unsigned long long *s, int r) {
  Bits<W> b;
#pragma unroll
  for (int k = 0; k < W; ++k) b.w[k] = s[r * W + k];
  return b;
}
template <int W>
__device__ __forceinline__ Bits<W> band(Bits<W> a, Bits<W> b) {
#pragma unroll
  for (int k = 0; k < W; ++k) a.w[k] &= b.w[k];
  return a;
}
template <int W>
__device__ __forceinline__ Bits<W> bor(Bits<W> a, Bits<W> b) {
#pragma unroll
  for (int k = 0; k < W; ++k) a.w[k] |= b.w[k];
  return a;
}
template <int W>
__device__ __forceinline__ Bits<W> bandnot(Bits<W> a, Bits<W> b) {
#pragma unroll
  for (int k = 0; k < W; ++k) a.w[k] &= ~b.w[k];
  return a;
}
template <int W>
__device__ __forceinline__ Bits<W> bzero() {
  Bits<W> a;
#pragma unroll
  for (int k = 0; k < W; ++k) a.w[k] = 0ull;
  return a;
}
template <int W>
__device__ __forceinline__ bool bany(Bits<W> a) {
  unsigned long long r = 0;
#pragma unroll
  for (int k = 0; k < W; ++k) r |= a.w[k];
  return r != 0ull;
}
template <int W>
__device__ __forceinline__ int bpop(Bits<W> a) {
  int r = 0;
#pragma unroll
  for (int k = 0; k < W; ++k) r += __popcll(a.w[k]);
  return r;
}
// Word k of a bitset is selected by comparisons, never by a computed
// index (that would put the words in scratch memory).
template <int W>
__device__ __forceinline__ bool btest(Bits<W> a, int v) {
  unsigned long long word = a.w[0];
#pragma unroll
  for (int k = 1; k < W; ++k)
    if ((v >> 6) == k) word = a.w[k];
  return (word >> (v & 63)) & 1ull;
}
template <int W>
__device__ __forceinline__ Bits<W> bsingle(int v) {
  Bits<W> a;
#pragma unroll
  for (int k = 0; k < W; ++k) a.w[k] = (W == 1 || (v >> 6) == k) ? 1ull << (v & 63) : 0ull;
  return a;
}
// Lowest set bit index (a must be non-empty); clears it.
template <int W>
__device__ __forceinline__ int bpop_lowest(Bits<W> &a) {
  if (W <= 2) {
    if (W == 1 || a.w[0]) {
      const int v = __ffsll((long long)a.w[0]) - 1;
      a.w[0] &= a.w[0] - 1ull;
      return v;
    }
    const int v = __ffsll((long long)a.w[W - 1]) - 1;
    a.w[W - 1] &= a.w[W - 1] - 1ull;
    return 64 + v;
  }
  // first non-empty word, picked and rewritten by comparisons
  int k = W - 1;
#pragma unroll
  for (int j = W - 2; j >= 0; --j)
    if (a.w[j]) k = j;
  unsigned long long word = a.w[0];
#pragma unroll
  for (int j = 1; j < W; ++j)
    if (k == j) word = a.w[j];
  const int v = __ffsll((long long)word) - 1;
  const unsigned long long rest = word & (word - 1ull);
#pragma unroll
  for (int j = 0; j < W; ++j)
    if (k == j) a.w[j] = rest;
  return 64 * k + v;
}
// {w : w <= u}
template <int W>
__device__ __forceinline__ Bits<W> low_through(int u) {
  Bits<W> a;
#pragma unroll
  for (int k = 0; k < W; ++k) {
    const int b = u - 64 * k;  // bits of word k at or below u: b + 1, clamped
    a.w[k] = b >= 63 ? ~0ull : (b < 0 ? 0ull : ((2ull << b) - 1ull));
  }
  return a;
}

// End vertices of a frontier path: v1 | vt << 8 in 16 bits up to 256
// vertices, v1 | vt << 16 in 32 bits beyond.
template <int W>
__device__ __forceinline__ unsigned vv_load(const Frontier &f, unsigned long long e) {
  if constexpr (CC_BIG(W)) return f.vw[e];
  else return (unsigned)f.vv[e];
}
template <int W>
__device__ __forceinline__ void vv_store(const Frontier &f, unsigned long long e, int v1, int vt) {
  if constexpr (CC_BIG(W)) f.vw[e] = (unsigned)v1 | ((unsigned)vt << 16);
  else f.vv[e] = (unsigned short)(v1 | (vt << 8));
}
template <int W>
__device__ __forceinline__ int vv_v1(unsigned x) {
  return CC_BIG(W) ? (int)(x & 0xffffu) : (int)(x & 0xffu);
}
template <int W>
__device__ __forceinline__ int vv_vt(unsigned x) {
  return CC_BIG(W) ? (int)(x >> 16) : (int)(x >> 8);
}

// ------------------------------------------------------- wave primitives
__device__ __forceinline__ int lane_id() { return __lane_id(); }

// (the builtin takes the predicate as a lane mask, as compares produce it)
__device__ __forceinline__ unsigned long long wave_ballot(bool p) {
  return __builtin_amdgcn_ballot_w64(p);
}

// Number of set bits of `mask` at lanes below this one.
__device__ __forceinline__ unsigned int lanes_below(unsigned long long mask) {
  return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

// Sum over a fully active wavefront by data-parallel moves, the same
// pattern as wave_min_u32 below (butterflies within rows, then row
// broadcasts), returned to every lane from lane 63.
__device__ __forceinline__ unsigned wave_sum_u32_full(unsigned v) {
  v += (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0xb1, 0xf, 0xf, false);
  v += (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x4e, 0xf, 0xf, false);
  v += (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xf, 0xf, false);
  v += (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xf, 0xf, false);
  v += (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);
  v += (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);
  return (unsigned)__builtin_amdgcn_readlane((int)v, CC_WAVE - 1);
}
__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, CC_WAVE);
  return v;
}
// Minimum over the wavefront by data-parallel primitives (cross-lane moves
// inside the vector ALU, no LDS round trip): within quads, half-rows and
// rows of 16 lanes, then row 0 into row 1 and row 2 into row 3, then the
// lower half into the upper; lane 63 ends with the minimum, which is
// returned to every lane.  Lanes a move does not write keep the identity.
// The whole wavefront must be active.
__device__ __forceinline__ unsigned wave_min_u32(unsigned v) {
  const int id = -1;  // 0xffffffff
  v = min(v, (unsigned)__builtin_amdgcn_update_dpp(id, (int)v, 0xb1, 0xf, 0xf, false));   // quad 1,0,3,2
  v = min(v, (unsigned)__builtin_amdgcn_update_dpp(id, (int)v, 0x4e, 0xf, 0xf, false));   // quad 2,3,0,1
  v = min(v, (unsigned)__builtin_amdgcn_update_dpp(id, (int)v, 0x141, 0xf, 0xf, false));  // half-row mirror
  v = min(v, (unsigned)__builtin_amdgcn_update_dpp(id, (int)v, 0x140, 0xf, 0xf, false));  // row mirror
  v = min(v, (unsigned)__builtin_amdgcn_update_dpp(id, (int)v, 0x142, 0xa, 0xf, false));  // row bcast 15
  v = min(v, (unsigned)__builtin_amdgcn_update_dpp(id, (int)v, 0x143, 0xc, 0xf, false));  // row bcast 31
  return (unsigned)__builtin_amdgcn_readlane((int)v, CC_WAVE - 1);
}

// A value every lane of the wavefront holds, moved to scalar registers.
__device__ __forceinline__ unsigned uni_u32(unsigned v) {
  return (unsigned)__builtin_amdgcn_readfirstlane((int)v);
}
__device__ __forceinline__ unsigned long long uni_u64(unsigned long long v) {
  return (unsigned long long)uni_u32((unsigned)v) |
         ((unsigned long long)uni_u32((unsigned)(v >> 32)) << 32);
}
// Room left in a shard of cap_s slots after `base` of them are taken,
// clamped to 32 bits (a wavefront writes fewer than 2^32 per step).
__device__ __forceinline__ unsigned room_after(unsigned long long base, unsigned long long cap_s) {
  const unsigned long long r = base < cap_s ? cap_s - base : 0ull;
  return r > 0xffffffffull ? 0xffffffffu : (unsigned)r;
}

template <typename T>
__device__ __forceinline__ T ld_acquire(T *p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
// Plain read of a value written by an earlier kernel on the same stream
// (kernel boundaries already order it); no cache maintenance.
template <typename T>
__device__ __forceinline__ T ld_relaxed(T *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_release(T *p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Coherent single accesses (relaxed, agent scope): each is one sc1 load or
// store, with no cache-wide maintenance.  Relaxed accesses order nothing
// else: a payload written with them is published by a release fence before
// its flag is stored (release_agent) and read after an acquire fence that
// follows the load which saw the flag (acquire_agent); on gfx950 these are
// the L2 write-back and invalidate that make the payload visible to the
// other XCDs.
template <typename T>
__device__ __forceinline__ T ld_coh(T *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_coh(T *p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Waits until every memory access this wavefront issued has completed.
__device__ __forceinline__ void wait_mem() { __builtin_amdgcn_s_waitcnt(0); }
// Called by the whole wavefront: every lane's earlier stores are visible
// at agent scope before any later store of the wavefront (the flag).
__device__ __forceinline__ void release_agent() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }
// Called by the whole wavefront after the load that saw the flag.
__device__ __forceinline__ void acquire_agent() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }

// Records a failed consistency check of the depth-first kernel (the run
// reports an error instead of using the value).
__device__ __forceinline__ void dfs_corrupt(CcCtl *ctl, unsigned kind, unsigned value) {
  atomicOr(&ctl->status, CC_DEV_CORRUPT);
  atomicCAS(&ctl->diag, 0u, (kind << 24) | (value & 0xffffffu));
}

// A word for the host: the store, then a system-scope release so the line
// leaves the GPU caches now rather than at some later write-back.
__device__ __forceinline__ void st_system(unsigned int *p, unsigned int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
}

// ------------------------------------------------------------ shards
// The value of another lane by a data-parallel move (both halves moved the
// same way); lanes the move does not write, or whose source lane is out of
// range, get 0.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ unsigned long long dpp_u64(unsigned long long x) {
  const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)x, CTRL, ROW_MASK,
                                                            0xf, false);
  const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(x >> 32), CTRL,
                                                            ROW_MASK, 0xf, false);
  return ((unsigned long long)hi << 32) | lo;
}
// Wavefront-wide inclusive scan of one value per lane (lane = shard); writes
// pre[0] = 0 and pre[s + 1] = sum of shards 0..s.  Called by a whole
// (fully active) wavefront.
__device__ __forceinline__ void shard_prefix(unsigned long long v, unsigned long long *pre) {
  const int lane = lane_id();
  // inclusive scan: shifts by 1, 2, 4, 8 within rows of 16 lanes, then
  // row 0's total into row 1 and row 2's into row 3, then rows 0-1's total
  // (lane 31) into rows 2 and 3
  unsigned long long x = v;
  x += dpp_u64<0x111, 0xf>(x);
  x += dpp_u64<0x112, 0xf>(x);
  x += dpp_u64<0x114, 0xf>(x);
  x += dpp_u64<0x118, 0xf>(x);
  x += dpp_u64<0x142, 0xa>(x);
  x += dpp_u64<0x143, 0xc>(x);
  pre[lane + 1] = x;
  if (lane == 0) pre[0] = 0ull;
}

// Shard holding global element i (0 <= i < pre[CC_SHARDS]): the largest s
// with pre[s] <= i, which is never an empty shard.
__device__ __forceinline__ int shard_of(const unsigned long long *pre, unsigned long long i) {
  int lo = 0, hi = CC_SHARDS;
#pragma unroll
  for (int it = 0; it < 6; ++it) {
    const int mid = (lo + hi) >> 1;
    if (pre[mid] <= i) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Lane l's value of v, in scalar registers (l uniform).
__device__ __forceinline__ unsigned long long lane_u64(unsigned long long v, int l) {
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v >> 32), l);
  return ((unsigned long long)hi << 32) | lo;
}

// For a wavefront whose lanes hold the consecutive indices b + lane (b
// uniform), with lane s holding end = pre[s + 1]: when one shard holds all
// of b .. b+63, sets `base` so that index b + lane is element base + lane
// of the sharded array (cap_s per shard) and returns true; otherwise the
// lanes look their shards up one by one (shard_of).  Called by a whole
// wavefront.
__device__ __forceinline__ bool run_in_one_shard(unsigned long long end, unsigned long long b,
                                                 unsigned long long cap_s,
                                                 unsigned long long &base) {
  const int s = (int)__popcll(wave_ballot(end <= b));  // shards ending at or before b
  if (s >= CC_SHARDS) return false;
  if (b + CC_WAVE > lane_u64(end, s)) return false;
  const unsigned long long p = lane_u64(end, s > 0 ? s - 1 : 0);
  base = (unsigned long long)s * cap_s + b - (s > 0 ? p : 0ull);
  return true;
}

// -------------------------------------------------------------- decoding
// Writes the k vertices of a chordless cycle given as a bitset C over
// original ids: it starts at the smallest id and continues towards the
// smaller of that vertex's two cycle neighbours.  In an induced cycle every
// vertex has exactly two neighbours inside C, so the walk is unique.
// sNo holds the adjacency rows in original-id space.
template <int W>
__device__ void write_cycle(const unsigned long long *sNo, Bits<W> C, int k, int *dst) {
  Bits<W> it = C;
  const int start = bpop_lowest(it);
  Bits<W> nb = band(row<W>(sNo, start), C);
  const int first = bany(nb) ? bpop_lowest(nb) : start;  // C is always a cycle here
  dst[0] = start;
  dst[1] = first;
  if constexpr (CC_BIG(W)) {
    // Rows in device memory: walk from both ends at once (positions 2, 3,
    // ... from the smaller neighbour, k-2, k-3, ... from the other one), so
    // the chain of dependent row loads is half as long.
    const int last = bany(nb) ? bpop_lowest(nb) : start;
    if (k > 2) dst[k - 1] = last;
    int fp = start, fc = first, bp = start, bc = last;
    for (int i = 2, j = k - 2; i <= j; ++i, --j) {
      Bits<W> nf = band(row<W>(sNo, fc), bandnot(C, bsingle<W>(fp)));
      Bits<W> nbk = band(row<W>(sNo, bc), bandnot(C, bsingle<W>(bp)));
      const int fn = bany(nf) ? bpop_lowest(nf) : start;
      const int bn = bany(nbk) ? bpop_lowest(nbk) : start;
      dst[i] = fn;
      if (j != i) dst[j] = bn;
      fp = fc;
      fc = fn;
      bp = bc;
      bc = bn;
    }
  } else {
    int prev = start, cur = first;
    for (int j = 2; j < k; ++j) {
      Bits<W> nx = band(row<W>(sNo, cur), bandnot(C, bsingle<W>(prev)));
      const int nxt = bany(nx) ? bpop_lowest(nx) : start;
      dst[j] = nxt;
      prev = cur;
      cur = nxt;
    }
  }
}

// Where cycle `cyc` (global output index) of length k with vertices at
// global offset `pos` goes in the caller's buffers: shifted into the
// output window; false if the cycle is outside the window or the buffers.
__device__ __forceinline__ bool out_slot(const OutDev &out, int k, long long &cyc,
                                         long long &pos) {
  if (k < out.kmin || k > out.kmax) return false;
  cyc -= out.cshift;
  pos -= out.vshift;
  return cyc >= 0 && pos >= 0 && cyc < out.cyc_cap && pos + k <= out.verts_cap;
}

// ----------------------------------------------------------------- zero
// The control block before a run on a graph of cols - 2 vertices: the
// per-shard counters in the columns the run uses, everything after them.
__device__ __forceinline__ void zero_ctl_body(CcCtl *ctl, int cols, size_t tid, size_t nt) {
  for (size_t i = tid; i < (size_t)CC_SHARDS * cols; i += nt) {
    const size_t s = i / cols, k = i - s * cols;
    ctl->count_sh[s][k] = 0ull;
    ctl->hist_sh[s][k] = 0ull;
  }
  unsigned int *rest = (unsigned int *)&ctl->cum_c[0];
  const size_t words = (sizeof(CcCtl) - offsetof(CcCtl, cum_c)) / 4;
  for (size_t i = tid; i < words; i += nt) rest[i] = 0u;
}

__global__ void k_zero(unsigned int *p, size_t words) {
  size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < words; i += stride) p[i] = 0u;
}

// --------------------------------------------------------------- ingest
// The ingest's result for a host spinning on mapped memory: the status word
// and the pairs bound, a system-scope release, then the ready word.
__device__ void ingest_reply(unsigned int *reply, unsigned int st, long long pairs) {
  __hip_atomic_store(reply + 1, st, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  __hip_atomic_store(reply + 2, (unsigned)(unsigned long long)pairs, __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_SYSTEM);
  __hip_atomic_store(reply + 3, (unsigned)((unsigned long long)pairs >> 32), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_SYSTEM);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
  st_system(reply, 1u);
}

// One block per graph.  Validates the CSR (simple, symmetric), builds the
// adjacency bitsets, computes the degree labelling (Section 2: repeatedly
// take the remaining vertex of minimum remaining degree, smallest id on
// ties; it gets the next label) with one wavefront holding W vertices per
// lane, and writes the bitsets renumbered by label plus the original ones.
template <int W>
__global__ __launch_bounds__(128) void k_ingest(const int *__restrict__ graph_vtx_off,
                                                int n_single, const int *__restrict__ rp,
                                                const int *__restrict__ ci,
                                                unsigned long long *__restrict__ adj_out,
                                                unsigned long long *__restrict__ adj_orig,
                                                int *__restrict__ perm_out,
                                                int *__restrict__ label_out,
                                                unsigned int *__restrict__ status,
                                                long long *__restrict__ bound,
                                                unsigned int *reply) {
  __shared__ unsigned long long sA[CC_ROWS(W) * W];
  __shared__ int sLab[CC_ROWS(W)];
  __shared__ unsigned int sErr;
  __shared__ unsigned int sDeg;
  __shared__ unsigned long long sPairs;
  const int g = blockIdx.x;
  const int tid = threadIdx.x;
  int v0 = 0, n = n_single;
  if (graph_vtx_off) {
    v0 = graph_vtx_off[g];
    n = graph_vtx_off[g + 1] - v0;
  }
  if (tid == 0) {
    sErr = 0u;
    sDeg = 0u;
    sPairs = 0ull;
  }
  for (int i = tid; i < CC_ROWS(W) * W; i += blockDim.x) sA[i] = 0ull;
  __syncthreads();
  if (n < 0 || n > 64 * W) {
    if (tid == 0) {
      status[g] = CC_DEV_NOT_SIMPLE;
      if (reply) ingest_reply(reply, CC_DEV_NOT_SIMPLE, 0);
    }
    return;
  }
  const long long e0 = rp[v0];
  const long long eN = rp[v0 + n];
  const bool bad_head = (v0 == 0 && e0 != 0) || eN < e0 || (eN - e0) > (long long)n * (n - 1);
  if (bad_head) {
    // an invalid graph keeps no edges, so later stages find nothing in it
    for (int i = tid; i < n * W; i += blockDim.x) adj_out[(size_t)v0 * W + i] = 0ull;
    // every thread took this branch from the same two loads; once all have
    // made them the host may free the CSR, so the reply waits for them
    __syncthreads();
    if (tid == 0) {
      status[g] = CC_DEV_NOT_SIMPLE;
      if (reply) ingest_reply(reply, CC_DEV_NOT_SIMPLE, 0);
    }
    return;
  }
  for (int v = tid; v < n; v += blockDim.x) {
    const long long a = rp[v0 + v], b = rp[v0 + v + 1];
    if (b < a || a < e0 || b > eN) {
      atomicOr(&sErr, CC_DEV_NOT_SIMPLE);
      continue;
    }
    Bits<W> r = bzero<W>();
    bool bad = false;
    // four neighbour ids in flight per round
    for (long long e = a; e < b && !bad; e += 4) {
      int w4[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) w4[k] = e + k < b ? ci[e + k] - v0 : -1;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (e + k >= b || bad) continue;
        const int w = w4[k];
        if (w < 0 || w >= n || w == v) {
          bad = true;
        } else {
          bad = btest(r, w);
          r = bor(r, bsingle<W>(w));
        }
      }
    }
    if (bad) atomicOr(&sErr, CC_DEV_NOT_SIMPLE);
#pragma unroll
    for (int k = 0; k < W; ++k) sA[v * W + k] = r.w[k];
    atomicMax(&sDeg, (unsigned)(b - a));
    atomicAdd(&sPairs, (unsigned long long)((b - a) * (b - a - 1) / 2));
  }
  __syncthreads();
  // symmetry: w in N(v) implies v in N(w)
  for (int v = tid; v < n; v += blockDim.x) {
    Bits<W> r = row<W>(sA, v);
    while (bany(r)) {
      int w = bpop_lowest(r);
      if (!btest(row<W>(sA, w), v)) atomicOr(&sErr, CC_DEV_NOT_SIMPLE);
    }
  }
  __syncthreads();
  if (sErr) {
    for (int i = tid; i < n * W; i += blockDim.x) adj_out[(size_t)v0 * W + i] = 0ull;
    if (tid == 0) {
      status[g] = sErr;
      if (reply) ingest_reply(reply, sErr, 0);
    }
    return;
  }
  if constexpr (CC_BIG(W)) {
    if (tid < CC_WAVE) {
      // lane holds vertices tid + 64 j, j < W; key = degree << 10 | id
      // picks the minimum degree, then the smallest id.  The rows stay in
      // LDS: removing u reads u's row once (the same words for every lane),
      // and vertex tid + 64 j is bit tid of its word j.
      int deg[W];
      bool alive[W];
#pragma unroll
      for (int j = 0; j < W; ++j) {
        const int v = tid + CC_WAVE * j;
        alive[j] = v < n;
        deg[j] = alive[j] ? bpop(row<W>(sA, v)) : 0;
      }
      for (int i = 0; i < n; ++i) {
        unsigned mine = 0xffffffffu;
#pragma unroll
        for (int j = 0; j < W; ++j)
          if (alive[j]) mine = min(mine, ((unsigned)deg[j] << 10) | (unsigned)(tid + CC_WAVE * j));
        const unsigned key = wave_min_u32(mine);
        const int u = (int)(key & 0x3ffu);
#pragma unroll
        for (int j = 0; j < W; ++j) {
          const int v = tid + CC_WAVE * j;
          if (v == u) {
            alive[j] = false;
            sLab[u] = i;
          }
          if (alive[j] && ((sA[u * W + j] >> tid) & 1ull)) --deg[j];
        }
      }
    }
  } else if (tid < CC_WAVE) {
    // lane holds vertices tid + 64 j, j < W; key = degree << 8 | id picks
    // the minimum degree, then the smallest id
    int deg[W];
    bool alive[W];
    Bits<W> nb[W];  // the lane's rows, kept in registers for all rounds
#pragma unroll
    for (int j = 0; j < W; ++j) {
      const int v = tid + CC_WAVE * j;
      alive[j] = v < n;
      nb[j] = alive[j] ? row<W>(sA, v) : bzero<W>();
      deg[j] = bpop(nb[j]);
    }
    for (int i = 0; i < n; ++i) {
      unsigned mine = 0xffffffffu;
#pragma unroll
      for (int j = 0; j < W; ++j)
        if (alive[j]) mine = min(mine, ((unsigned)deg[j] << 8) | (unsigned)(tid + CC_WAVE * j));
      const unsigned key = wave_min_u32(mine);
      const int u = (int)(key & 0xffu);
#pragma unroll
      for (int j = 0; j < W; ++j) {
        const int v = tid + CC_WAVE * j;
        if (v == u) {
          alive[j] = false;
          sLab[u] = i;
        }
        if (alive[j] && btest(nb[j], u)) --deg[j];
      }
    }
  }
  __syncthreads();
  for (int v = tid; v < n; v += blockDim.x) {
    const int l = sLab[v];
    perm_out[v0 + l] = v;
    label_out[v0 + v] = l;
    Bits<W> r = row<W>(sA, v);
#pragma unroll
    for (int k = 0; k < W; ++k) adj_orig[(size_t)(v0 + v) * W + k] = r.w[k];
    Bits<W> out = bzero<W>();
    while (bany(r)) out = bor(out, bsingle<W>(sLab[bpop_lowest(r)]));
#pragma unroll
    for (int k = 0; k < W; ++k) adj_out[(size_t)(v0 + l) * W + k] = out.w[k];
  }
  if (tid == 0) {
    status[g] = 0x100u | (sDeg << 16);  // bit 8: ok; bits 16..: max degree
    if (bound) bound[g] = (long long)sPairs;
    if (reply) ingest_reply(reply, 0x100u | (sDeg << 16), (long long)sPairs);
  }
}

// ------------------------------------------------------------- stage one
// Initial triplets and triangles (Algorithm 1's set T(G) and the triangles
// of C; Algorithm 2 computes the same sets).  One block; each thread takes
// (u, x) pairs with x a higher-labelled neighbour of u and scans the
// neighbours y of u above x.  Results are numbered with LDS counters and
// dealt round-robin over the shards (item j -> shard j % CC_SHARDS, slot
// j / CC_SHARDS), so every shard gets the same share.
// Stage one on a block of T threads, with the graph already in LDS (sN,
// sPerm) and *sTrip = *sTri = 0 before the call.  Writes the triplets to f
// and, enumerating, the triangles to st; sets the counters and the state of
// step 0.  Ends with a barrier; *sTrip and *sTri then hold the totals.
// With a range of roots (rr.lo > 0 or rr.hi < LLONG_MAX) every root (u, x,
// y) gets its index in the order of u's original id, then x's, then y's
// (ctl->root_base[u] holds the index of u's first root): the pairs of
// higher-labelled neighbours x' of u that come before x by original id
// each contribute their own higher-labelled partners, and y is ranked among
// x's partners by original id.  Only roots inside the range are kept.
template <int W, bool ENUM, int T>
__device__ void triplets_body(const GraphDev &g, CcCtl *ctl, const Frontier &f, const Stage &st,
                              const unsigned long long *sN, const int *sPerm,
                              unsigned int *sTrip, unsigned int *sTri, const RootRange rr) {
  const int n = g.n;
  const int tid = threadIdx.x;
  const bool ranged = rr.lo > 0 || rr.hi < 0x7fffffffffffffffll;
  // (u, x) pairs: all n^2 of them spread over the block when the rows are
  // in LDS; beyond 256 vertices (rows in device memory) one thread per u,
  // walking u's higher-labelled neighbours x
  int u = 0, x = -1;
  Bits<W> nu = bzero<W>(), xs = bzero<W>();
  [[maybe_unused]] int idx = tid;
  if (CC_BIG(W)) u = tid - T;  // the first call below moves to u = tid
  while (true) {
    if constexpr (CC_BIG(W)) {
      while (!bany(xs)) {
        u += T;
        if (u >= n) break;
        nu = row<W>(sN, u);
        xs = bandnot(nu, low_through<W>(u));
      }
      if (u >= n) break;
      x = bpop_lowest(xs);
    } else {
      if (idx >= n * n) break;
      u = idx / n;
      x = idx - u * n;
      idx += T;
      nu = row<W>(sN, u);
      if (x <= u || !btest(nu, x)) continue;
    }
    const Bits<W> nx = row<W>(sN, x);
    const Bits<W> ys0 = bandnot(nu, low_through<W>(x));
    long long base = 0;
    if (ranged) {
      const Bits<W> up = bandnot(nu, low_through<W>(u));  // neighbours above u
      base = ctl->root_base[u];
      Bits<W> it = up;
      while (bany(it)) {
        const int xp = bpop_lowest(it);
        if (sPerm[xp] < sPerm[x]) base += bpop(bandnot(up, low_through<W>(xp)));
      }
    }
    Bits<W> ys = ys0;
    while (bany(ys)) {
      const int y = bpop_lowest(ys);
      if (ranged) {
        long long ix = base;
        Bits<W> it = ys0;
        while (bany(it)) {
          const int yp = bpop_lowest(it);
          ix += sPerm[yp] < sPerm[y] ? 1 : 0;
        }
        if (ix < rr.lo || ix >= rr.hi) continue;
      }
      if (btest(nx, y)) {
        const unsigned j = atomicAdd(sTri, 1u);
        if (ENUM) {
          const unsigned long long slot = (j % CC_SHARDS) * st.cap_s + j / CC_SHARDS;
          if (j / CC_SHARDS < st.cap_s) {
            const Bits<W> C =
                bor(bor(bsingle<W>(sPerm[x]), bsingle<W>(sPerm[u])), bsingle<W>(sPerm[y]));
#pragma unroll
            for (int k = 0; k < W; ++k) st.C[k * st.cap + slot] = C.w[k];
          }
        }
      } else {
        const unsigned j = atomicAdd(sTrip, 1u);
        if (j / CC_SHARDS < f.cap_s) {
          const unsigned long long slot = (j % CC_SHARDS) * f.cap_s + j / CC_SHARDS;
          const Bits<W> X = bor(nu, low_through<W>(u));
#pragma unroll
          for (int k = 0; k < W; ++k) f.X[k * f.cap + slot] = X.w[k];
          if (ENUM) {
            const Bits<W> S =
                bor(bor(bsingle<W>(sPerm[x]), bsingle<W>(sPerm[u])), bsingle<W>(sPerm[y]));
#pragma unroll
            for (int k = 0; k < W; ++k) f.S[k * f.cap + slot] = S.w[k];
          }
          vv_store<W>(f, slot, x, y);
        }
      }
    }
  }
  __syncthreads();
  const unsigned trip = *sTrip, tri = *sTri;
  if (tid < CC_SHARDS) {
    const unsigned s = tid;
    ctl->count_sh[s][3] = trip > s ? (trip - s + CC_SHARDS - 1) / CC_SHARDS : 0u;
    ctl->hist_sh[s][3] = tri > s ? (tri - s + CC_SHARDS - 1) / CC_SHARDS : 0u;
  }
  if (tid == 0) {
    // step 0 expands the triplets (frontier buffer 1) and, enumerating,
    // decodes the triangles (stage pair 0, slot 0)
    StepState S{};
    S.t = 3;
    S.fbuf = 1;
    S.spair = 0;
    S.slen0 = ENUM ? 3 : 0;
    S.step = 0;
    ctl->ss[1] = S;  // for step launch 1, unless the head kernel goes on
  }
  __syncthreads();
}

// Number of stage-one roots (triangles and initial triplets): the sum over
// vertices of C(d+, 2), d+ = neighbours with a higher label.  One block.
template <int W>
__global__ __launch_bounds__(CC_BLOCK) void k_root_total(GraphDev g, long long *out) {
  __shared__ unsigned long long sum;
  if (threadIdx.x == 0) sum = 0ull;
  __syncthreads();
  for (int l = threadIdx.x; l < g.n; l += CC_BLOCK) {
    const unsigned long long dp = (unsigned long long)bpop(bandnot(row<W>(g.adj, l), low_through<W>(l)));
    if (dp > 1) atomicAdd(&sum, dp * (dp - 1) / 2);
  }
  __syncthreads();
  if (threadIdx.x == 0) *out = (long long)sum;
}

template <int W>
__global__ __launch_bounds__(CC_BLOCK) void k_triplets_batch(BatchDev bt) {
  __shared__ unsigned long long sN[CC_ROWS(W) * W];
  __shared__ unsigned int sTrip, sTri;
  const int g = bt.g0 + blockIdx.x;
  const int tid = threadIdx.x;
  const int vo = bt.vtx_off[g];
  const int n = bt.vtx_off[g + 1] - vo;
  const unsigned long long base = (unsigned long long)bt.root_off[g];
  const unsigned long long slots = (unsigned long long)(bt.root_off[g + 1] - bt.root_off[g]);
  for (int i = tid; i < n * W; i += CC_BLOCK) sN[i] = bt.adj[(size_t)vo * W + i];
  if (tid == 0) {
    sTrip = 0u;
    sTri = 0u;
  }
  __syncthreads();
  for (int idx = tid; idx < n * n; idx += CC_BLOCK) {
    const int u = idx / n, x = idx - u * n;
    const Bits<W> nu = row<W>(sN, u);
    if (x <= u || !btest(nu, x)) continue;
    const Bits<W> nx = row<W>(sN, x);
    Bits<W> ys = bandnot(nu, low_through<W>(x));
    while (bany(ys)) {
      const int y = bpop_lowest(ys);
      if (btest(nx, y)) {
        atomicAdd(&sTri, 1u);
      } else {
        const unsigned j = atomicAdd(&sTrip, 1u);
        if (j < slots) {
          const unsigned long long e = base + j;
          const Bits<W> X = bor(nu, low_through<W>(u));
#pragma unroll
          for (int k = 0; k < W; ++k) bt.rX[k * bt.rcap + e] = X.w[k];
          bt.rvv[e] = (unsigned short)(x | (y << 8));
          bt.rgid[e] = (unsigned)g;
        }
      }
    }
  }
  __syncthreads();
  for (unsigned long long j = sTrip + tid; j < slots; j += CC_BLOCK) bt.rgid[base + j] = CC_NO_GRAPH;
  if (tid == 0 && sTri) atomicAdd(&bt.hist[(size_t)g * bt.hist_stride + 3], (unsigned long long)sTri);
}

// ------------------------------------------------------ breadth-first steps
// Algorithm 3 over the frontier of open paths, one step at a time.  A step
// expands the paths with t vertices either by one level (extensions with
// t+1 vertices, closures = cycles with t+1 vertices) or, when its output
// provably fits, by two: each lane follows its path's extensions one more
// level itself, so the paths with t+1 vertices are counted but never
// written, and closures with t+1 and t+2 vertices are both found.  A step
// also decodes the cycles the previous step staged.
//
// Expansion: a block takes chunks of CC_BLOCK * CC_LEVEL_IPT consecutive
// paths (one lane per path, CC_LEVEL_IPT rounds; CC_LEVEL_IPT_W4 with
// four-word bitsets, whose larger lane state favours fewer); each wavefront
// counts what its lanes produce, reserves room for it with one atomic per
// counter on the block's shard, and ranks its lanes inside the reserved
// ranges with ballot/mbcnt, so the stores of a round land on consecutive
// slots.  Closures are counted in hist_sh[.][k] and, when enumerating,
// staged as vertex bitsets for the next step to decode.
//
// Decoding: cycle g of length k (global order: shards in turn) goes to
// output index cum_c[k-1] + g, vertices at cum_v[k-1] + g * k, so the output
// is ordered by length.  Every lane decodes one cycle.
//
// The steps run as one launch each (k_step; Algorithm 4's fixed relaunches,
// without readback: the step's t and buffers live in CcCtl).

// Shared memory of one block running steps.
template <int W, bool ENUM>
struct LevelLds {
  // label-space and original-id adjacency (beyond 256 vertices the rows are
  // read from device memory instead)
  unsigned long long N[CC_BIG(W) ? 1 : CC_ROWS(W) * W];
  unsigned long long No[ENUM && !CC_BIG(W) ? CC_ROWS(W) * W : 1];
  int Perm[ENUM ? CC_ROWS(W) : 1];
  unsigned long long Pre[CC_SHARDS + 1];
  unsigned long long PreH0[ENUM ? CC_SHARDS + 1 : 1];
  unsigned long long PreH1[ENUM ? CC_SHARDS + 1 : 1];
  unsigned int WaveA[CC_BLOCK / CC_WAVE];   // count mode: closures one level down
  unsigned int WaveB[CC_BLOCK / CC_WAVE];   // count mode: closures two levels down
  unsigned long long Cum[2];
  unsigned long long PrevFront;
  int Flags;      // written by wave 0: the input frontier overflowed
  int FlagsH[2];  // written by waves 1 and 2: a staged length overflowed
  // per-wavefront buffer of decoded cycles (vertex ids, cycle after cycle)
  int Dec[ENUM ? CC_BLOCK / CC_WAVE : 1][ENUM ? CC_DEC_WORDS : 1];
  unsigned long long Tot[CC_ROWS(W) + 2];  // per-length totals (the step that ends the loop)
};

// step_body results
#define CC_LEVEL_NEXT 0      // the step expanded its paths; continue
#define CC_LEVEL_SWITCH 1    // handed over to the depth-first kernel
#define CC_LEVEL_EMPTY 2     // no paths left: the loop is over

template <int W, bool ENUM>
__device__ void load_graph_lds(const GraphDev &g, LevelLds<W, ENUM> &L) {
  if (!CC_BIG(W))
    for (int i = threadIdx.x; i < g.n * W; i += CC_BLOCK) L.N[i] = g.adj[i];
  if (ENUM) {
    if (!CC_BIG(W))
      for (int i = threadIdx.x; i < g.n * W; i += CC_BLOCK) L.No[i] = g.adj_orig[i];
    for (int i = threadIdx.x; i < g.n; i += CC_BLOCK) L.Perm[i] = g.perm[i];
  }
}

// Field-wise selection (a select of whole structs would go through scratch).
__device__ __forceinline__ Frontier pick(bool c, const Frontier &a, const Frontier &b) {
  Frontier f;
  f.X = c ? a.X : b.X;
  f.S = c ? a.S : b.S;
  f.vv = c ? a.vv : b.vv;
  f.vw = c ? a.vw : b.vw;
  f.cap = c ? a.cap : b.cap;
  f.cap_s = c ? a.cap_s : b.cap_s;
  return f;
}
__device__ __forceinline__ Stage pick(bool c, const Stage &a, const Stage &b) {
  Stage s;
  s.C = c ? a.C : b.C;
  s.cap = c ? a.cap : b.cap;
  s.cap_s = c ? a.cap_s : b.cap_s;
  return s;
}

// Reservations of four counts per wavefront: every lane adds its counts,
// lane 0 reserves room for the wavefront's totals on the shard's counters,
// and the bases come back in scalar registers.  No block barrier: each
// wavefront goes on as soon as its own atomics return.  Called by a whole
// (fully active) wavefront.
__device__ __forceinline__ void reserve(unsigned a, unsigned b, unsigned c, unsigned d,
                                        unsigned long long *ctrA, unsigned long long *ctrB,
                                        unsigned long long *ctrC, unsigned long long *ctrD,
                                        unsigned long long &baseA, unsigned long long &baseB,
                                        unsigned long long &baseC, unsigned &wa, unsigned &wb,
                                        unsigned &wc) {
  wa = wave_sum_u32_full(a);
  wb = wave_sum_u32_full(b);
  wc = wave_sum_u32_full(c);
  const unsigned wd = wave_sum_u32_full(d);
  unsigned long long ba = 0, bb = 0, bc = 0;
  if (lane_id() == 0) {
    if (wa && ctrA) ba = atomicAdd(ctrA, (unsigned long long)wa);
    if (wb && ctrB) bb = atomicAdd(ctrB, (unsigned long long)wb);
    if (wc && ctrC) bc = atomicAdd(ctrC, (unsigned long long)wc);
    if (wd && ctrD) atomicAdd(ctrD, (unsigned long long)wd);
  }
  baseA = lane_u64(ba, 0);
  baseB = lane_u64(bb, 0);
  baseC = lane_u64(bc, 0);
}

// Orders this wavefront's LDS accesses before and after (a wavefront's LDS
// operations complete in order; this keeps the compiler from moving them).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Decodes the h staged cycles of length k from stage st (shard prefix pre):
// cycle gi goes to output index cb + gi, vertices at vb + gi * k.  Wavefront
// gw of nwg takes runs of `per` consecutive cycles: each lane walks one
// cycle into the wavefront's LDS buffer, then the run's vertex range, which
// is contiguous in the output, is written by consecutive lanes.
template <int W, bool ENUM>
__device__ void decode_run(const unsigned long long *No, int *buf, const Stage &st,
                           const unsigned long long *pre, unsigned long long h, int k,
                           long long cb, long long vb, const OutDev &out, unsigned long long gw,
                           unsigned long long nwg) {
  if (h == 0 || k < 3 || k < out.kmin || k > out.kmax) return;
  cb -= out.cshift;  // into the output window
  vb -= out.vshift;
  const int lane = lane_id();
  // each lane's cycle at an odd stride in buf, so the lanes' stores of one
  // position fall in distinct LDS banks
  const int sk = k | 1;
  const unsigned long long per = (unsigned long long)min(CC_WAVE, CC_DEC_WORDS / sk);
  const float rk = 1.0f / (float)k;
  const unsigned long long end = pre[lane + 1];
  for (unsigned long long g0 = gw * per; g0 < h; g0 += nwg * per) {
    const unsigned long long nb = min(per, h - g0);
    const unsigned long long gi = g0 + (unsigned long long)lane;
    unsigned long long rb = 0;
    const bool one = run_in_one_shard(end, g0, st.cap_s, rb);
    if ((unsigned long long)lane < nb) {
      unsigned long long e;
      if (one) {
        e = rb + (unsigned long long)lane;
      } else {
        const int s = shard_of(pre, gi);
        e = (unsigned long long)s * st.cap_s + (gi - pre[s]);
      }
      Bits<W> C;
#pragma unroll
      for (int w = 0; w < W; ++w) C.w[w] = st.C[w * st.cap + e];
      write_cycle<W>(No, C, k, buf + lane * sk);
      const long long cyc = cb + (long long)gi;
      const long long pos = vb + (long long)gi * k;
      if (cyc >= 0 && pos >= 0 && cyc < out.cyc_cap && pos + k <= out.verts_cap)
        out.offs[cyc] = pos;
    }
    wave_lds_sync();
    const long long base = vb + (long long)g0 * k;
    const int words = (int)nb * k;
    for (int d = lane; d < words; d += CC_WAVE) {
      // word d is position d mod k of the run's cycle d / k; the quotient
      // by a float reciprocal is exact: (d + 1/2) / k lies at least 1/(2k)
      // from an integer, and the product's relative error (~2^-23) moves it
      // by less than d/k * 2^-23, far less for d < CC_DEC_WORDS
      const int c = (int)(((float)d + 0.5f) * rk);
      const int j = d - c * k;
      const long long q = base + d;
      if (q >= 0 && q < out.verts_cap) out.verts[q] = buf[c * sk + j];
    }
    wave_lds_sync();  // the next run overwrites buf
  }
}

// The state of a step, written by block 0 of the launch before, so that a
// plain load sees it (a launch's writes are visible to the launches after it
// on the stream).  The same holds for the counters a step starts from: plain
// loads are served by each XCD's L2 after one miss, where loads at agent
// scope would take every block of the grid to memory for the same few lines.
__device__ __forceinline__ StepState load_state(const StepState *p) { return *p; }

// One step for this block.  Every block of the grid reads the same state
// and counters and so reaches the same result.  With lds_ready false the
// graph is loaded into LDS here, together with the counters.
template <int W, bool ENUM>
__device__ int step_body(const GraphDev &g, CcCtl *ctl, const LevelBufs &B, const OutDev &out,
                         int step, const StepState &S, StepState *next, int forced_level,
                         int maxc, bool allow_two, LevelLds<W, ENUM> &L, bool lds_ready) {
  constexpr int IPT = CC_BIG(W) ? CC_LEVEL_IPT_BIG : W == 4 ? CC_LEVEL_IPT_W4 : CC_LEVEL_IPT;
  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int wave = tid / CC_WAVE;
  // the adjacency rows: in LDS, or in device memory beyond 256 vertices
  const unsigned long long *const Nr = CC_BIG(W) ? g.adj : L.N;
  const unsigned long long *const Nor = CC_BIG(W) ? g.adj_orig : L.No;
  if (S.done) return CC_LEVEL_EMPTY;
  const int t = S.t;
  const int n = g.n;
  const Frontier fin = pick(S.fbuf != 0, B.f[1], B.f[0]);
  const Frontier fout = pick(S.fbuf != 0, B.f[0], B.f[1]);
  const int p = S.spair, q = 1 - S.spair;  // stage pairs: decoded here, written here
  const Stage sd0 = pick(p != 0, B.st[2], B.st[0]), sd1 = pick(p != 0, B.st[3], B.st[1]);
  const Stage sw0 = pick(q != 0, B.st[2], B.st[0]), sw1 = pick(q != 0, B.st[3], B.st[1]);
  // Each wavefront issues all its loads before it uses any of them, so that
  // their latencies overlap: the shard counters (wave 0: paths with t
  // vertices, waves 1 and 2: the staged cycles to decode, wave 3: the
  // previous step's children, paths with t-1 vertices), the cumulative
  // output offsets, and the graph rows.
  const int kh = wave == 1 ? S.slen0 : S.slen1;  // waves 1 and 2: staged length
  unsigned long long c = 0, cum0 = 0, cum1 = 0;
  if (wave == 0) {
    c = ctl->count_sh[lane][t];
    if (ENUM && S.slen0) {
      cum0 = ctl->cum_c[S.slen0 - 1];
      cum1 = ctl->cum_v[S.slen0 - 1];
    }
  } else if (wave == 1 || wave == 2) {
    if (ENUM && kh) c = ctl->hist_sh[lane][kh];
  } else if (wave == 3 && S.prev_two) {
    c = ctl->count_sh[lane][t - 1];
  }
  if (!lds_ready) load_graph_lds<W, ENUM>(g, L);
  if (wave == 0) {
    shard_prefix(c, L.Pre);
    const unsigned long long mo = wave_ballot(c > fin.cap_s);
    if (lane == 0) {
      L.Flags = mo ? 1 : 0;
      L.Cum[0] = cum0;
      L.Cum[1] = cum1;
    }
  } else if (wave == 1 || wave == 2) {
    // each of these waves writes its own flag every step
    bool ovf = false;
    if (ENUM && kh) {
      shard_prefix(c, wave == 1 ? L.PreH0 : L.PreH1);
      ovf = wave_ballot(c > (wave == 1 ? sd0.cap_s : sd1.cap_s)) != 0ull;
    }
    if (lane == 0) L.FlagsH[wave - 1] = ovf ? 2 : 0;
  } else if (wave == 3 && S.prev_two) {
    const unsigned long long tot = wave_sum_u64(c);
    if (lane == 0) L.PrevFront = tot;
  }
  __syncthreads();
  const int flags = L.Flags | L.FlagsH[0] | L.FlagsH[1];
  const unsigned long long cnt = L.Pre[CC_SHARDS];
  const unsigned vblk = blockIdx.x, vgrid = gridDim.x;
  const unsigned long long shard_end = L.Pre[lane + 1];  // lane s: end of input shard s
  if (blockIdx.x == 0 && tid == 0) {
    if (step < CC_HSLOTS) ctl->step_level[step] = t;
    if (S.prev_two) ctl->front[t - 1] = L.PrevFront;
  }

  // ---- decode the cycles the previous step staged (lengths slen0, slen1)
  if (ENUM && S.slen0 && !(flags & 2)) {
    const int k0 = S.slen0, k1 = S.slen1;
    const unsigned long long h0 = L.PreH0[ENUM ? CC_SHARDS : 0],
                             h1 = k1 ? L.PreH1[ENUM ? CC_SHARDS : 0] : 0ull;
    const long long cb0 = (long long)L.Cum[0], vb0 = (long long)L.Cum[1];
    const long long cb1 = cb0 + (long long)h0, vb1 = vb0 + (long long)h0 * k0;
    // The decode counts blocks from the far end of the grid, the expansion
    // below from the start: when either has little work, the two run on
    // different blocks at the same time instead of one after the other.
    constexpr int NWB = CC_BLOCK / CC_WAVE;
    const unsigned long long gw = (unsigned long long)(vgrid - 1 - vblk) * NWB + wave;
    const unsigned long long nwg = (unsigned long long)vgrid * NWB;
    decode_run<W, ENUM>(Nor, L.Dec[ENUM ? wave : 0], sd0, L.PreH0, h0, k0, cb0, vb0, out, gw, nwg);
    decode_run<W, ENUM>(Nor, L.Dec[ENUM ? wave : 0], sd1, L.PreH1, h1, k1, cb1, vb1, out, gw, nwg);
    if (blockIdx.x == 0 && tid == 0) {
      ctl->cum_c[k0] = (unsigned long long)cb1;
      ctl->cum_v[k0] = (unsigned long long)vb1;
      if (k1) {
        ctl->cum_c[k1] = (unsigned long long)(cb1 + (long long)h1);
        ctl->cum_v[k1] = (unsigned long long)(vb1 + (long long)h1 * k1);
      }
    }
  }

  // ---- hand over to the depth-first kernel when needed
  int sw_level = 0, sw_skip = 0, sw_max = 0, sw_buf = 0;
  if (flags & 3) {
    // Only a one-level step can overflow (a two-level step is taken only
    // when its output fits), so the paths with t-1 vertices it expanded are
    // still intact in the other buffer.
    if (S.prev_two) {
      if (blockIdx.x == 0 && tid == 0) dfs_corrupt(ctl, CC_DIAG_PATH, (unsigned)t);
      return CC_LEVEL_EMPTY;
    }
    sw_level = t - 1;
    sw_buf = 1 - S.fbuf;
    if (flags & 2) {
      // The previous step staged more cycles than fit: its paths are handed
      // over again and everything from them on is recounted.
      sw_skip = CC_SKIP_FRONT;
      sw_max = t - 1;
    } else {
      // The previous step produced more paths than fit: its closures and
      // path count are already recorded.
      sw_skip = CC_SKIP_FRONT | CC_SKIP_CLOSE;
      sw_max = t;
    }
  } else if (t == forced_level) {
    sw_level = t;
    sw_buf = S.fbuf;
    sw_skip = 0;
    sw_max = t;
  }
  StepState N = S;
  N.done = 1;
  N.step = step + 1;
  if (sw_level) {
    if (blockIdx.x == 0 && tid == 0) {
      ctl->skip = sw_skip;
      ctl->switch_level = sw_level;
      ctl->bfs_max_len = sw_max;
      ctl->root_buf = sw_buf;
      *next = N;
      __threadfence();
      st_release(&ctl->mode, 1);
    }
    return CC_LEVEL_SWITCH;
  }
  if (cnt == 0) {
    if (blockIdx.x == 0 && tid == 0) *next = N;
    return CC_LEVEL_EMPTY;
  }

  // ---- one level or two
  // Paths per lane per chunk: up to IPT, fewer when the frontier is small,
  // so that a small step spreads over more blocks instead of making a few
  // lanes walk several paths one after the other.
  const unsigned long long grid = vgrid;
  const int ipt = (int)min((unsigned long long)IPT,
                           max(1ull, (cnt + grid * CC_BLOCK - 1) / (grid * CC_BLOCK)));
  const unsigned long long chunk = (unsigned long long)CC_BLOCK * ipt;
  // No shard takes the output of more than per_shard input paths (a block
  // writes to shard blockIdx mod CC_SHARDS).
  const unsigned long long per_shard =
      (cnt + grid * chunk - 1) / (grid * chunk) * chunk * ((grid + CC_SHARDS - 1) / CC_SHARDS);
  const unsigned long long mc = (unsigned long long)(maxc > 1 ? maxc : 1);
  const bool two = allow_two && t + 2 <= n && t + 1 != forced_level &&
                   per_shard * mc * mc <= fout.cap_s &&
                   (!ENUM || per_shard * mc * mc <= sw1.cap_s);
  if (blockIdx.x == 0 && tid == 0) {
    N.t = t + (two ? 2 : 1);
    N.fbuf = 1 - S.fbuf;
    N.spair = q;
    N.slen0 = ENUM ? t + 1 : 0;
    N.slen1 = (ENUM && two) ? t + 2 : 0;
    N.prev_two = two ? 1 : 0;
    N.done = 0;
    *next = N;
    ctl->front[t] = cnt;
    atomicMax(&ctl->peak, cnt);
  }
  // Blocks without a chunk have nothing more to do in this step.
  if ((unsigned long long)vblk * chunk >= cnt) return CC_LEVEL_NEXT;
  const int osh = blockIdx.x % CC_SHARDS;  // this block's output shard
  unsigned long long acc1 = 0, acc2 = 0;   // closures (count mode)
  for (unsigned long long c0 = (unsigned long long)vblk * chunk; c0 < cnt; c0 += grid * chunk) {
    Bits<W> X[IPT], Sv[IPT];
    int v1[IPT], vt[IPT];
    bool valid[IPT];
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
      const unsigned long long wb =
          c0 + (unsigned long long)j * CC_BLOCK + (unsigned long long)wave * CC_WAVE;
      const unsigned long long i = wb + (unsigned long long)lane;
      valid[j] = j < ipt && i < cnt;
      X[j] = bzero<W>();
      Sv[j] = bzero<W>();
      v1[j] = 0;
      vt[j] = 0;
      unsigned long long rb = 0;
      const bool one = run_in_one_shard(shard_end, wb, fin.cap_s, rb);
      if (valid[j]) {
        unsigned long long e;
        if (one) {
          e = rb + (unsigned long long)lane;
        } else {
          const int s = shard_of(L.Pre, i);
          e = (unsigned long long)s * fin.cap_s + (i - L.Pre[s]);
        }
#pragma unroll
        for (int w = 0; w < W; ++w) X[j].w[w] = fin.X[w * fin.cap + e];
        if (ENUM) {
#pragma unroll
          for (int w = 0; w < W; ++w) Sv[j].w[w] = fin.S[w * fin.cap + e];
        }
        const unsigned vv = vv_load<W>(fin, e);
        v1[j] = vv_v1<W>(vv);
        vt[j] = vv_vt<W>(vv);
      }
    }
    // counts: a = paths written, b = closures one level down, c = closures
    // two levels down, d = children of a two-level step
    unsigned ca = 0, cb = 0, cc = 0, cd = 0;
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
      if (!valid[j]) continue;
      const Bits<W> nvt = row<W>(Nr, vt[j]), nv1 = row<W>(Nr, v1[j]);
      const Bits<W> cand = bandnot(nvt, X[j]);
      cb += (unsigned)bpop(band(cand, nv1));
      Bits<W> ext = bandnot(cand, nv1);
      if (!two) {
        ca += (unsigned)bpop(ext);
      } else {
        cd += (unsigned)bpop(ext);
        const Bits<W> Xc = bor(X[j], nvt);
        while (bany(ext)) {
          const Bits<W> cand2 = bandnot(row<W>(Nr, bpop_lowest(ext)), Xc);
          cc += (unsigned)bpop(band(cand2, nv1));
          ca += (unsigned)bpop(bandnot(cand2, nv1));
        }
      }
    }
    const int kA = two ? t + 2 : t + 1;  // length of the paths written
    unsigned long long baseA, baseB, baseC;
    unsigned wa, wb, wc;
    reserve(ca, cb, cc, cd, &ctl->count_sh[osh][kA], ENUM ? &ctl->hist_sh[osh][t + 1] : nullptr,
            (ENUM && two) ? &ctl->hist_sh[osh][t + 2] : nullptr,
            two ? &ctl->count_sh[osh][t + 1] : nullptr, baseA, baseB, baseC, wa, wb, wc);
    if (!ENUM) {
      acc1 += cb;
      acc2 += cc;
    }
    // ---- write the paths (extensions, or grandchildren)
    // Each output range is addressed from a wavefront-uniform pointer to its
    // first slot in shard osh plus a 32-bit rank; ranks at or beyond the
    // shard's room are dropped (the next step sees the overflow).
    if (wa) {
      const unsigned long long b0 = min(baseA, fout.cap_s);
      const unsigned room = room_after(baseA, fout.cap_s);
      unsigned long long *const Xo = fout.X + (unsigned long long)osh * fout.cap_s + b0;
      unsigned long long *const So = fout.S + (unsigned long long)osh * fout.cap_s + b0;
      const unsigned long long vo0 = (unsigned long long)osh * fout.cap_s + b0;
      unsigned off = 0;
#pragma unroll
      for (int j = 0; j < IPT; ++j) {
        const Bits<W> nvt = row<W>(Nr, vt[j]), nv1 = row<W>(Nr, v1[j]);
        const Bits<W> Xc = bor(X[j], nvt);
        Bits<W> ext = valid[j] ? bandnot(bandnot(nvt, X[j]), nv1) : bzero<W>();
        // lane iterator: current child c and its remaining extensions cur
        Bits<W> cur = two ? bzero<W>() : ext, Xg = Xc;
        int c = -1;
        while (true) {
          if (two) {
            while (!bany(cur) && bany(ext)) {
              c = bpop_lowest(ext);
              const Bits<W> nc = row<W>(Nr, c);
              cur = bandnot(bandnot(nc, Xc), nv1);
              Xg = bor(Xc, nc);
            }
          }
          const bool has = bany(cur);
          const unsigned long long mask = wave_ballot(has);
          if (!mask) break;
          if (has) {
            const int v = bpop_lowest(cur);
            const unsigned r = off + lanes_below(mask);
            if (r < room) {
#pragma unroll
              for (int w = 0; w < W; ++w) Xo[w * fout.cap + r] = Xg.w[w];
              if (ENUM) {
                Bits<W> Sn = bor(Sv[j], bsingle<W>(L.Perm[v]));
                if (two) Sn = bor(Sn, bsingle<W>(L.Perm[c]));
#pragma unroll
                for (int w = 0; w < W; ++w) So[w * fout.cap + r] = Sn.w[w];
              }
              vv_store<W>(fout, vo0 + r, v1[j], v);
            }
          }
          off += (unsigned)__popcll(mask);
        }
      }
    }
    // ---- stage the closures (enumerate mode)
    if (ENUM && wb) {
      const unsigned room = room_after(baseB, sw0.cap_s);
      unsigned long long *const Co =
          sw0.C + (unsigned long long)osh * sw0.cap_s + min(baseB, sw0.cap_s);
      unsigned off = 0;
#pragma unroll
      for (int j = 0; j < IPT; ++j) {
        const Bits<W> nvt = row<W>(Nr, vt[j]), nv1 = row<W>(Nr, v1[j]);
        Bits<W> cl = valid[j] ? band(bandnot(nvt, X[j]), nv1) : bzero<W>();
        while (true) {
          const bool has = bany(cl);
          const unsigned long long mask = wave_ballot(has);
          if (!mask) break;
          if (has) {
            const int v = bpop_lowest(cl);
            const unsigned r = off + lanes_below(mask);
            if (r < room) {
              const Bits<W> C = bor(Sv[j], bsingle<W>(L.Perm[v]));
#pragma unroll
              for (int w = 0; w < W; ++w) Co[w * sw0.cap + r] = C.w[w];
            }
          }
          off += (unsigned)__popcll(mask);
        }
      }
    }
    if (ENUM && wc) {
      const unsigned room = room_after(baseC, sw1.cap_s);
      unsigned long long *const Co =
          sw1.C + (unsigned long long)osh * sw1.cap_s + min(baseC, sw1.cap_s);
      unsigned off = 0;
#pragma unroll
      for (int j = 0; j < IPT; ++j) {
        const Bits<W> nvt = row<W>(Nr, vt[j]), nv1 = row<W>(Nr, v1[j]);
        const Bits<W> Xc = bor(X[j], nvt);
        Bits<W> ext = valid[j] ? bandnot(bandnot(nvt, X[j]), nv1) : bzero<W>();
        Bits<W> cur = bzero<W>();
        int c = -1;
        while (true) {
          while (!bany(cur) && bany(ext)) {
            c = bpop_lowest(ext);
            cur = band(bandnot(row<W>(Nr, c), Xc), nv1);
          }
          const bool has = bany(cur);
          const unsigned long long mask = wave_ballot(has);
          if (!mask) break;
          if (has) {
            const int v = bpop_lowest(cur);
            const unsigned r = off + lanes_below(mask);
            if (r < room) {
              const Bits<W> C =
                  bor(bor(Sv[j], bsingle<W>(L.Perm[c])), bsingle<W>(L.Perm[v]));
#pragma unroll
              for (int w = 0; w < W; ++w) Co[w * sw1.cap + r] = C.w[w];
            }
          }
          off += (unsigned)__popcll(mask);
        }
      }
    }
  }
  if (!ENUM) {
    acc1 = wave_sum_u64(acc1);
    acc2 = wave_sum_u64(acc2);
    if (lane == 0) {
      L.WaveA[wave] = (unsigned)acc1;  // per-wavefront closures fit 32 bits per step
      L.WaveB[wave] = (unsigned)acc2;
    }
    __syncthreads();
    if (tid == 0) {
      unsigned long long s1 = 0, s2 = 0;
      for (int w = 0; w < CC_BLOCK / CC_WAVE; ++w) {
        s1 += L.WaveA[w];
        s2 += L.WaveB[w];
      }
      if (s1) atomicAdd(&ctl->hist_sh[osh][t + 1], s1);
      if (s2) atomicAdd(&ctl->hist_sh[osh][t + 2], s2);
    }
  }
  return CC_LEVEL_NEXT;
}

// Per-length cycle totals: lengths up to bfs_max_len come from the
// breadth-first levels (summed over shards); longer ones, when the
// depth-first kernel took over in enumerate mode, from its counting pass.
// Count mode accumulates everything in the shards.  One block; sTot has
// `slots` entries, at least n + 2 (all of CC_HSLOTS when the depth-first
// kernel may have counted).  bfs_only: the caller knows the depth-first
// kernel did not take over.
__device__ void length_totals(CcCtl *ctl, int n, bool enumerate, unsigned long long *sTot,
                              int slots = CC_HSLOTS, bool bfs_only = false) {
  const int tid = threadIdx.x;
  for (int k = tid; k < slots; k += blockDim.x) sTot[k] = 0ull;
  __syncthreads();
  const bool dfs = !bfs_only && ld_relaxed(&ctl->mode) != 0;
  // a run on n vertices uses the columns 0..n+1 (the only ones zeroed)
  const int kmax = min((enumerate && dfs) ? ctl->bfs_max_len : CC_HSLOTS - 1, n + 1);
  // the shard counters of the used columns, several loads in flight per
  // thread before their sums go into LDS
  constexpr int PER = 16;
  const int cols = max(kmax + 1, 0), total = CC_SHARDS * cols;
  for (int base = tid; base < total; base += blockDim.x * PER) {
    unsigned long long v[PER];
    int kk[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int p = base + j * (int)blockDim.x;
      kk[j] = -1;
      v[j] = 0ull;
      if (p < total) {
        const int s = p / cols;
        kk[j] = p - s * cols;
        v[j] = ld_relaxed(&ctl->hist_sh[s][kk[j]]);
      }
    }
#pragma unroll
    for (int j = 0; j < PER; ++j)
      if (kk[j] >= 0 && v[j]) atomicAdd(&sTot[kk[j]], v[j]);
  }
  __syncthreads();
  if (enumerate && dfs)
    for (int k = tid; k < slots; k += blockDim.x)
      if (k > kmax) sTot[k] = ctl->dfs_hist[k];
  __syncthreads();
}

// Final histogram (ctl->hist; entries from `slots` on stay as zeroed); in
// enumerate mode also closes the offsets array with the total vertex count.
// One block, sTot as for length_totals.
__device__ void finalize_body(CcCtl *ctl, const OutDev &out, int n, bool enumerate,
                              unsigned long long *sTot, int slots, bool bfs_only = false) {
  length_totals(ctl, n, enumerate, sTot, slots, bfs_only);
  for (int k = threadIdx.x; k < slots; k += blockDim.x) ctl->hist[k] = sTot[k];
  if (enumerate && threadIdx.x == 0) {
    // the closing offset of the output window
    long long c = 0, v = 0;
    for (int k = 0; k <= n && k < slots; ++k) {
      if (k < out.kmin || k > out.kmax) continue;
      c += (long long)sTot[k];
      v += (long long)sTot[k] * k;
    }
    if (c <= out.cyc_cap && v <= out.verts_cap && out.offs) out.offs[c] = v;
  }
}

// --------------------------------------------------------- one-block head
// Stage one and the leading levels on one block of CC_HEAD_BLOCK(W) threads,
// with the frontier in LDS: two buffers of `cap` paths in dynamic shared
// memory (X words, S words when enumerating, then vv), used in turn.  Each
// level takes one pass to count every path's extensions and closures, a
// block-wide scan for exact offsets, and one pass to write the extensions
// to the other buffer and each closure's cycle straight to the output
// (cycles of one length come from one level, so their output range is
// known).  Nothing is staged and no global counter is touched, so a level
// costs a few LDS round trips and barriers.
//
// The head stops at the first level whose paths do not fit (or at the
// forced depth-first level): it writes that level's paths to frontier
// buffer 0, dealt round-robin over the shards, with the counters, the
// cumulative output offsets and the state of step launch 1 (ss[1]).  If
// the frontier empties first, the loop is over (ss[1] says done).  Launch 0
// for host_done.
template <int W, bool ENUM>
struct HeadLds {
  // rows in LDS up to 256 vertices (beyond, the head reads them from
  // device memory)
  unsigned long long N[CC_BIG(W) ? 1 : CC_ROWS(W) * W];
  unsigned long long No[ENUM && !CC_BIG(W) ? CC_ROWS(W) * W : 1];
  int Perm[CC_ROWS(W)];
  unsigned long long WaveTot[CC_HEAD_THREADS / CC_WAVE];
  unsigned long long Front[CC_SLOTS(W)];  // paths expanded per length
  unsigned long long Hist[CC_SLOTS(W)];   // cycles found per length (above 3)
  unsigned int Trip, Tri;
  long long WCum[2];                    // wavefront phase results, for the block
  int WState[5];
};

// Head results of a run of levels on one wavefront
#define CC_HEAD_MORE 0   // the frontier outgrew the wavefront: back to the block
#define CC_HEAD_OVER 1   // the frontier emptied
#define CC_HEAD_STOP 2   // hand over at level t (forced level, or no room)

// The head's frontier buffer b (0 or 1) inside dynamic shared memory.
template <int W, bool ENUM>
struct HeadBuf {
  unsigned long long *X;
  unsigned long long *S;
  unsigned short *vv;  // end vertices v1 | vt << 8, up to 256 vertices
  unsigned int *vw;    // v1 | vt << 16 beyond
};
template <int W, bool ENUM>
__device__ __forceinline__ HeadBuf<W, ENUM> head_buf(unsigned long long *dyn, int cap, int b) {
  const int words = W * cap * (ENUM ? 2 : 1);
  const int per = words + (cap * (CC_BIG(W) ? 4 : 2) + 7) / 8;  // 8-byte words per buffer
  HeadBuf<W, ENUM> h;
  h.X = dyn + b * per;
  h.S = h.X + W * cap;
  h.vv = (unsigned short *)(h.X + words);
  h.vw = (unsigned int *)(h.X + words);
  return h;
}
template <int W, bool ENUM>
__device__ __forceinline__ unsigned hb_get(const HeadBuf<W, ENUM> &h, unsigned i) {
  if constexpr (CC_BIG(W)) return h.vw[i];
  else return (unsigned)h.vv[i];
}
template <int W, bool ENUM>
__device__ __forceinline__ void hb_put(const HeadBuf<W, ENUM> &h, unsigned i, int v1, int vt) {
  if constexpr (CC_BIG(W)) h.vw[i] = (unsigned)v1 | ((unsigned)vt << 16);
  else h.vv[i] = (unsigned short)(v1 | (vt << 8));
}

// Block-wide exclusive scan of two 32-bit counts packed in one 64-bit value
// (no carry between the halves: each half's total stays below 2^32).
// Returns this thread's offsets; *total receives the block's totals.
template <int NT>
__device__ __forceinline__ unsigned long long block_scan2(unsigned long long v,
                                                          unsigned long long *wave_tot,
                                                          unsigned long long *total) {
  constexpr int NW = NT / CC_WAVE;
  const int lane = lane_id(), wave = threadIdx.x / CC_WAVE;
  unsigned long long x = v;
#pragma unroll
  for (int o = 1; o < CC_WAVE; o <<= 1) {
    const unsigned long long y = __shfl_up(x, o, CC_WAVE);
    if (lane >= o) x += y;
  }
  if (lane == CC_WAVE - 1) wave_tot[wave] = x;
  __syncthreads();
  unsigned long long base = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    const unsigned long long t = wave_tot[w];
    if (w < wave) base += t;
    tot += t;
  }
  *total = tot;
  __syncthreads();  // wave_tot is reused by the next scan
  return base + x - v;
}

// Levels on one wavefront while the frontier has at most CC_WAVE paths, one
// path per lane: the same count / scan / write passes as the block, with
// the scan across lanes and no barrier (a wavefront's LDS operations
// complete in order).  Thin graphs (a long cycle, a wheel) spend every
// level here.  Updates t, cnt, b and the output cursors; returns
// CC_HEAD_MORE, CC_HEAD_OVER or CC_HEAD_STOP.
template <int W, bool ENUM>
__device__ int head_wave_levels(HeadLds<W, ENUM> &L, const unsigned long long *Nh,
                                const unsigned long long *Noh, unsigned long long *dyn, int cap,
                                int forced_level, const OutDev &out, int &t, unsigned &cnt,
                                int &b, long long &cum_c, long long &cum_v, int &odd) {
  const int lane = lane_id();
  while (true) {
    if (cnt == 0) return CC_HEAD_OVER;
    if (cnt > CC_WAVE) return CC_HEAD_MORE;
    if (t == forced_level || t + 2 >= CC_SLOTS(W)) return CC_HEAD_STOP;
    const HeadBuf<W, ENUM> cur = head_buf<W, ENUM>(dyn, cap, b);
    const HeadBuf<W, ENUM> nxt = head_buf<W, ENUM>(dyn, cap, 1 - b);
    const bool mine = (unsigned)lane < cnt;
    Bits<W> X = bzero<W>(), Sv = bzero<W>();
    unsigned vv = 0;
    if (mine) {
#pragma unroll
      for (int w = 0; w < W; ++w) X.w[w] = cur.X[w * cap + lane];
      if (ENUM) {
#pragma unroll
        for (int w = 0; w < W; ++w) Sv.w[w] = cur.S[w * cap + lane];
      }
      vv = hb_get<W, ENUM>(cur, lane);
    }
    const int vt = vv_vt<W>(vv), v1 = vv_v1<W>(vv);
    const Bits<W> nvt = row<W>(Nh, vt);
    const Bits<W> cand = mine ? bandnot(nvt, X) : bzero<W>();
    const Bits<W> n1 = row<W>(Nh, v1);
    Bits<W> ext = bandnot(cand, n1);
    Bits<W> cl = band(cand, n1);
    const unsigned long long v = (unsigned long long)bpop(ext) |
                                 ((unsigned long long)bpop(cl) << 32);
    unsigned long long x = v;
#pragma unroll
    for (int o = 1; o < CC_WAVE; o <<= 1) {
      const unsigned long long y = __shfl_up(x, o, CC_WAVE);
      if (lane >= o) x += y;
    }
    const unsigned long long tot = uni_u64(__shfl(x, CC_WAVE - 1, CC_WAVE));
    const unsigned te = (unsigned)tot, tc = (unsigned)(tot >> 32);
    if (te > (unsigned)cap) return CC_HEAD_STOP;
    unsigned oe = (unsigned)(x - v);
    unsigned long long oc = (x - v) >> 32;
    const Bits<W> Xn = bor(X, nvt);
    while (bany(ext)) {
      const int u = bpop_lowest(ext);
#pragma unroll
      for (int w = 0; w < W; ++w) nxt.X[w * cap + oe] = Xn.w[w];
      if (ENUM) {
        const Bits<W> Sn = bor(Sv, bsingle<W>(L.Perm[u]));
#pragma unroll
        for (int w = 0; w < W; ++w) nxt.S[w * cap + oe] = Sn.w[w];
      }
      hb_put<W, ENUM>(nxt, oe, v1, u);
      ++oe;
    }
    if (ENUM) {
      while (bany(cl)) {
        const int u = bpop_lowest(cl);
        long long idx = cum_c + (long long)oc;
        long long pos = cum_v + (long long)oc * (t + 1);
        if (out_slot(out, t + 1, idx, pos)) {
          write_cycle<W>(Noh, bor(Sv, bsingle<W>(L.Perm[u])), t + 1, out.verts + pos);
          out.offs[idx] = pos;
        }
        ++oc;
      }
    }
    if (lane == 0) {
      L.Front[t] = cnt;
      L.Hist[t + 1] = tc;
    }
    if (tc && ((t + 1) & 1)) odd = 1;
    wave_lds_sync();
    cum_c += tc;
    cum_v += (long long)tc * (t + 1);
    cnt = te;
    b = 1 - b;
    ++t;
  }
}

template <int W, bool ENUM>
__global__ __launch_bounds__(CC_HEAD_BLOCK(W)) void k_head(GraphDev g, CcCtl *ctl, LevelBufs B,
                                                          OutDev out, int forced_level,
                                                          int cap_lds, unsigned int *host_done,
                                                          int zero_cols, RootRange rr) {
  constexpr int T = CC_HEAD_BLOCK(W);
  __shared__ HeadLds<W, ENUM> L;
  extern __shared__ unsigned long long dyn[];
  const int tid = threadIdx.x;
  const int n = g.n;
  if (host_done && tid == 0)
    __hip_atomic_store(host_done + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  // the run's control block, as k_zero_ctl (the barrier below orders these
  // stores before this block's later use of it; later kernels follow in
  // stream order)
  if (zero_cols > 0) zero_ctl_body(ctl, zero_cols, tid, T);
  if (!CC_BIG(W)) {
    for (int i = tid; i < n * W; i += T) L.N[i] = g.adj[i];
    if (ENUM)
      for (int i = tid; i < n * W; i += T) L.No[i] = g.adj_orig[i];
  }
  // the rows: in LDS up to 256 vertices, in device memory beyond
  const unsigned long long *const Nh = CC_BIG(W) ? g.adj : L.N;
  const unsigned long long *const Noh = CC_BIG(W) ? g.adj_orig : L.No;
  for (int i = tid; i < n; i += T) L.Perm[i] = g.perm[i];
  for (int k = tid; k < CC_SLOTS(W); k += T) {
    L.Front[k] = 0ull;
    L.Hist[k] = 0ull;
  }
  if (tid == 0) {
    L.Trip = 0u;
    L.Tri = 0u;
  }
  __syncthreads();
  if (rr.lo > 0 || rr.hi < 0x7fffffffffffffffll) {
    // the index of each vertex's first root: prefix over original ids of
    // C(d+, 2), d+ = neighbours with a higher label
    for (int l = tid; l < n; l += T) ctl->orig_label[L.Perm[l]] = l;
    __syncthreads();
    if (tid == 0) {
      long long acc = 0;
      for (int v = 0; v < n; ++v) {
        const int l = ctl->orig_label[v];
        const long long dp = bpop(bandnot(row<W>(Nh, l), low_through<W>(l)));
        ctl->root_base[l] = acc;
        acc += dp * (dp - 1) / 2;
      }
    }
    __syncthreads();
  }
  // stage one, into the global buffers (frontier 1, stage 0)
  const Frontier f1 = B.f[1], f0 = B.f[0];
  const Stage st0 = B.st[0];
  // a hand-over deals at most cap paths over the shards of frontier 0
  const int cap = (int)min((unsigned long long)cap_lds, CC_SHARDS * f0.cap_s);
  triplets_body<W, ENUM, T>(g, ctl, f1, st0, Nh, L.Perm, &L.Trip, &L.Tri, rr);
  const unsigned trip = L.Trip, tri = L.Tri;
  int t = 3;
  unsigned cnt = trip;
  bool over = false;
  if (trip <= (unsigned)cap && forced_level != 3 && trip / CC_SHARDS < f1.cap_s) {
    // the triplets into LDS buffer 0 (this block wrote them: its barrier
    // orders those stores before these loads)
    HeadBuf<W, ENUM> cur = head_buf<W, ENUM>(dyn, cap, 0);
    for (unsigned j = tid; j < trip; j += T) {
      const unsigned long long e = (j % CC_SHARDS) * f1.cap_s + j / CC_SHARDS;
#pragma unroll
      for (int w = 0; w < W; ++w) cur.X[w * cap + j] = f1.X[w * f1.cap + e];
      if (ENUM) {
#pragma unroll
        for (int w = 0; w < W; ++w) cur.S[w * cap + j] = f1.S[w * f1.cap + e];
      }
      const unsigned x = vv_load<W>(f1, e);
      hb_put<W, ENUM>(cur, j, vv_v1<W>(x), vv_vt<W>(x));
    }
    // the triangles, written to the output at once
    long long cum_c = 0, cum_v = 0;
    if (ENUM) {
      for (unsigned j = tid; j < tri && j / CC_SHARDS < st0.cap_s; j += T) {
        const unsigned long long e = (j % CC_SHARDS) * st0.cap_s + j / CC_SHARDS;
        Bits<W> C;
#pragma unroll
        for (int w = 0; w < W; ++w) C.w[w] = st0.C[w * st0.cap + e];
        long long idx = j, pos = 3ll * j;
        if (out_slot(out, 3, idx, pos)) {
          write_cycle<W>(Noh, C, 3, out.verts + pos);
          out.offs[idx] = pos;
        }
      }
      cum_c = tri;
      cum_v = 3ll * tri;
    }
    __syncthreads();
    // the levels.  odd: a cycle of odd length has been found (a triangle
    // included); while none has, the graph looks bipartite.
    int b = 0, odd = tri != 0u;
    while (true) {
      if (cnt == 0) {
        over = true;
        break;
      }
      if (t == forced_level || t + 2 >= CC_SLOTS(W)) break;
      if (cnt <= CC_WAVE) {
        // small frontier: wavefront 0 alone, then tell the block
        if (tid < CC_WAVE) {
          const int r = head_wave_levels<W, ENUM>(L, Nh, Noh, dyn, cap, forced_level, out, t, cnt, b,
                                                  cum_c, cum_v, odd);
          if (tid == 0) {
            L.WState[0] = r;
            L.WState[1] = t;
            L.WState[2] = (int)cnt;
            L.WState[3] = b;
            L.WState[4] = odd;
            L.WCum[0] = cum_c;
            L.WCum[1] = cum_v;
          }
        }
        __syncthreads();
        const int r = L.WState[0];
        t = L.WState[1];
        cnt = (unsigned)L.WState[2];
        b = L.WState[3];
        odd = L.WState[4];
        cum_c = L.WCum[0];
        cum_v = L.WCum[1];
        __syncthreads();  // WState is rewritten by the next wavefront phase
        if (r == CC_HEAD_OVER) {
          over = true;
          break;
        }
        if (r == CC_HEAD_STOP) break;
        continue;
      }
      cur = head_buf<W, ENUM>(dyn, cap, b);
      const HeadBuf<W, ENUM> nxt = head_buf<W, ENUM>(dyn, cap, 1 - b);
      // count: extensions (low half) and closures (high half)
      unsigned long long mine = 0;
      for (unsigned i = tid; i < cnt; i += T) {
        Bits<W> X;
#pragma unroll
        for (int w = 0; w < W; ++w) X.w[w] = cur.X[w * cap + i];
        const unsigned vv = hb_get<W, ENUM>(cur, i);
        const Bits<W> cand = bandnot(row<W>(Nh, vv_vt<W>(vv)), X);
        const Bits<W> n1 = row<W>(Nh, vv_v1<W>(vv));
        mine += (unsigned long long)bpop(bandnot(cand, n1)) |
                ((unsigned long long)bpop(band(cand, n1)) << 32);
      }
      unsigned long long tot;
      const unsigned long long offs = block_scan2<T>(mine, L.WaveTot, &tot);
      const unsigned te = (unsigned)tot, tc = (unsigned)(tot >> 32);
      if (te > (unsigned)cap) break;  // the next level does not fit: hand over at t
      // In a graph that looks bipartite, every cycle has an even length.
      // Hand over at an odd length when the next level probably would not
      // fit anyway (te / cnt times te paths): the two-level steps from an
      // odd length then find every cycle one level down and never need the
      // walk for closures two levels down.
      if (!odd && (t & 1) && (unsigned long long)te * te > (unsigned long long)cap * cnt) break;
      unsigned oe = (unsigned)offs;
      unsigned long long oc = offs >> 32;
      for (unsigned i = tid; i < cnt; i += T) {
        Bits<W> X, Sv = bzero<W>();
#pragma unroll
        for (int w = 0; w < W; ++w) X.w[w] = cur.X[w * cap + i];
        if (ENUM) {
#pragma unroll
          for (int w = 0; w < W; ++w) Sv.w[w] = cur.S[w * cap + i];
        }
        const unsigned vv = hb_get<W, ENUM>(cur, i);
        const int vt = vv_vt<W>(vv), v1 = vv_v1<W>(vv);
        const Bits<W> nvt = row<W>(Nh, vt);
        const Bits<W> cand = bandnot(nvt, X);
        const Bits<W> n1 = row<W>(Nh, v1);
        Bits<W> ext = bandnot(cand, n1);
        const Bits<W> Xn = bor(X, nvt);
        while (bany(ext)) {
          const int v = bpop_lowest(ext);
#pragma unroll
          for (int w = 0; w < W; ++w) nxt.X[w * cap + oe] = Xn.w[w];
          if (ENUM) {
            const Bits<W> Sn = bor(Sv, bsingle<W>(L.Perm[v]));
#pragma unroll
            for (int w = 0; w < W; ++w) nxt.S[w * cap + oe] = Sn.w[w];
          }
          hb_put<W, ENUM>(nxt, oe, v1, v);
          ++oe;
        }
        if (ENUM) {
          Bits<W> cl = band(cand, n1);
          while (bany(cl)) {
            const int v = bpop_lowest(cl);
            long long idx = cum_c + (long long)oc;
            long long pos = cum_v + (long long)oc * (t + 1);
            if (out_slot(out, t + 1, idx, pos)) {
              write_cycle<W>(Noh, bor(Sv, bsingle<W>(L.Perm[v])), t + 1, out.verts + pos);
              out.offs[idx] = pos;
            }
            ++oc;
          }
        }
      }
      if (tid == 0) {
        L.Front[t] = cnt;
        L.Hist[t + 1] = tc;
      }
      if (tc && ((t + 1) & 1)) odd = 1;
      cum_c += tc;
      cum_v += (long long)tc * (t + 1);
      __syncthreads();
      cnt = te;
      b = 1 - b;
      ++t;
    }
    // Results and hand-over.  Steps 0 .. t-4 ran here, one level each.
    const int steps = t - 3;
    for (int k = 4 + tid; k <= t && k < CC_SLOTS(W); k += T)
      if (L.Hist[k]) ctl->hist_sh[0][k] = L.Hist[k];
    for (int k = 3 + tid; k < t; k += T) {
      ctl->front[k] = L.Front[k];
      ctl->step_level[k - 3] = k;
    }
    if (!over) {
      // this level's paths go to frontier buffer 0 for the step launches
      cur = head_buf<W, ENUM>(dyn, cap, b);
      for (unsigned i = tid; i < cnt; i += T) {
        const unsigned long long e = (i % CC_SHARDS) * f0.cap_s + i / CC_SHARDS;
#pragma unroll
        for (int w = 0; w < W; ++w) f0.X[w * f0.cap + e] = cur.X[w * cap + i];
        if (ENUM) {
#pragma unroll
          for (int w = 0; w < W; ++w) f0.S[w * f0.cap + e] = cur.S[w * cap + i];
        }
        const unsigned x = hb_get<W, ENUM>(cur, i);
        vv_store<W>(f0, e, vv_v1<W>(x), vv_vt<W>(x));
      }
      if (tid < CC_SHARDS)
        ctl->count_sh[tid][t] = cnt > (unsigned)tid ? (cnt - tid + CC_SHARDS - 1) / CC_SHARDS : 0u;
      if (tid == 0) {
        StepState S{};
        S.t = t;
        S.fbuf = 0;
        S.spair = 0;
        S.slen0 = 0;
        S.slen1 = 0;
        S.prev_two = 0;
        S.done = 0;
        S.step = steps;
        ctl->ss[1] = S;
        if (ENUM) {
          ctl->cum_c[t] = (unsigned long long)cum_c;
          ctl->cum_v[t] = (unsigned long long)cum_v;
        }
      }
    }
    if (tid == 0) {
      unsigned long long pk = 0;
      for (int k = 3; k < t; ++k) pk = max(pk, L.Front[k]);
      ctl->peak = max(pk, (unsigned long long)cnt);
      ctl->launch_step[1] = over ? 0 : steps + 1;
      if (over) {
        StepState S{};
        S.done = 1;
        ctl->ss[1] = S;
      }
      ctl->levels_run = steps;
      ctl->head_steps = steps;
      if (over && host_done) st_system(host_done, 1u);
    }
  } else if (tid == 0) {
    // too many triplets for LDS: the step launches start at step 0
    ctl->launch_step[1] = 1;
    ctl->levels_run = 0;
    ctl->head_steps = 0;
  }
}

// One launch per step (launch >= 1, after k_head): it runs the step whose
// state is in ss[launch] and writes the next launch's state (and, for the
// host's per-level timing, launch_step[launch + 1]).  host_done (pinned
// host memory, may be NULL): host_done[1] = launch + 1 when the launch
// starts, host_done[0] = launch + 1 when the loop is over, so the host
// stops launching and keeps few launches queued.
template <int W, bool ENUM>
__global__ __launch_bounds__(CC_BLOCK) void k_step(GraphDev g, CcCtl *ctl, LevelBufs B,
                                                   OutDev out, int launch, int forced_level,
                                                   int maxc, int allow_two,
                                                   unsigned int *host_done) {
  __shared__ LevelLds<W, ENUM> L;
  const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
  // this launch's state, written by the launch before it (the step index
  // travels in the state), and whether a launch before it handed over
  const StepState S = load_state(&ctl->ss[launch]);
  const int mode = ctl->mode;
  // the start mark for the host's pacing publishes nothing else, so it
  // needs no release (block 0 does not wait for it)
  if (host_done && lead)
    __hip_atomic_store(host_done + 1, (unsigned)launch + 1u, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_SYSTEM);
  const int step = S.step;
  StepState *next = &ctl->ss[launch + 1 < CC_HSLOTS ? launch + 1 : launch];
  if (mode != 0 || S.done || step < 0 || step >= g.n - 2) {
    // handed over, or queued after the loop ended: so is the next launch
    if (lead) {
      StepState D{};
      D.done = 1;
      *next = D;
      if (launch + 1 < CC_HSLOTS) ctl->launch_step[launch + 1] = 0;
      if (host_done) st_system(host_done, (unsigned)launch + 1u);
    }
    return;
  }
  const int r = step_body<W, ENUM>(g, ctl, B, out, step, S, next, forced_level, maxc,
                                   allow_two != 0, L, false);
  // The step that finds the frontier empty ends the run: block 0 (r is the
  // same for all its threads) also writes the final histogram and closing
  // offset, and host_done[3] tells the host to launch no finalize kernel.
  // (The levels ran to the end, so the depth-first kernel did not take over.)
  const bool fin = r == CC_LEVEL_EMPTY && blockIdx.x == 0 && host_done;
  if (fin) {
    __syncthreads();
    finalize_body(ctl, out, g.n, ENUM, L.Tot, CC_ROWS(W) + 2, true);
  }
  if (lead) {
    if (launch + 1 < CC_HSLOTS) ctl->launch_step[launch + 1] = r == CC_LEVEL_NEXT ? step + 2 : 0;
    ctl->levels_run = step + 1;
    if (r != CC_LEVEL_NEXT && host_done) {
      // host_done[2]: the loop handed over to the depth-first kernel;
      // host_done[3]: this launch finalized; both ordered before
      // host_done[0] by one release fence
      if (r == CC_LEVEL_SWITCH)
        __hip_atomic_store(host_done + 2, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      if (fin)
        __hip_atomic_store(host_done + 3, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
      __hip_atomic_store(host_done, (unsigned)launch + 1u, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
}

// ---------------------------------------------------------- depth-first
// Depth-first continuation (beyond the memory budget, on request, and for
// batches of small graphs).  The unit of work is a frame: the open paths
// <p, v> that share a prefix p, for every v in a set E of end vertices not
// expanded yet.  A frame holds their common exclusion set X, E, v1 and their
// length t (and, enumerating, the original ids S of p).  Expanding one of
// its paths takes the lowest v of E: the candidates N(v) \ X split into
// closures (adjacent to v1: chordless cycles of t + 1 vertices) and
// extensions, which form one new frame (X | N(v), the extensions, t + 1);
// the rest of E stays a frame of its own.  So every path costs the same
// constant work: one frame popped, at most two pushed.
//
// Each wavefront owns a LIFO stack of frames in two levels: its newest
// entries sit in a ring of C entries in LDS, older ones in device memory
// below them.  A step pops up to 64 frames (one per lane), expands one path
// of each and pushes the new frames back onto the LDS top, remainders below
// children, so the search goes depth first.  When the ring would overflow,
// its oldest entries move to device memory in whole-wavefront chunks; when
// it is empty, the next 64 frames come back from device memory.  Memory
// grows with depth, not with the frontier, and most steps touch LDS only.
// Work enters from the handed-over frontier (each path <q, vt> becomes the
// frame of q with E = {vt}), which wavefronts claim in private ranges (one
// atomic per range) and consume 64 at a time whenever their stack is empty.
//
// Load balance is by work requests through per-wavefront mailboxes (each
// wavefront polls only its own cache line, so no address is shared by the
// polling): an idle wavefront reads the published "frames I could give"
// hints of 64 others, asks the richest, and waits on its own line; a busy
// wavefront looks at its mailbox every few steps and either ships up to 64
// frames (the end of its private range, else the oldest, shallowest stack
// entries) into the requester's inbox or declines.  Payloads move with
// coherent single accesses and are published after an s_waitcnt, never with
// cache-wide fences.
//
// Termination: `busy` counts wavefronts that hold work, including work in
// transit (the donor counts the recipient before answering), so busy == 0
// with the handed-over frontier exhausted means no work is left anywhere.
// Cycle counts go to hist_out[(block % CC_SHARDS) * hist_stride + k].
//
// BATCH: many graphs at once.  Every frame carries its graph id; each
// wavefront keeps in LDS the adjacency rows of the graph its last
// single-graph step came from (one coalesced reload when a step's frames
// all belong to another graph; a step that mixes graphs reads its rows from
// device memory) and its share of that graph's histogram, which each lane
// adds its closures to and which goes to device memory when the wavefront
// moves to another graph or exits (a step that mixes graphs adds to the
// per-graph histograms directly, once per distinct (graph, length)); the
// handed-over paths are the batch's initial triplets in bt.r0..bt.r1,
// padding slots marked CC_NO_GRAPH.
//
// LDS per wavefront: the ring (X and E words, S words when enumerating, and
// one meta word: v1|t|root in the low half, the graph id of a batch in the
// high half) and, in batches, one graph's rows.  The ring holds 256 entries
// when an entry has at most 24 bytes, 128 up to 256 bytes, else 64 (graphs
// of more than 512 vertices); a step pops at most half of it (64 at most)
// and pushes at most twice what it popped.
template <int W, bool ENUM, bool BATCH>
struct DfsWaveLds {
  static constexpr int kEntry = 16 * W + (ENUM ? 8 * W : 0) + 8;
  static constexpr unsigned kC = kEntry <= 24 ? 256u : kEntry <= 256 ? 128u : 64u;
  // frames a step pops: a step pushes at most two per frame, which the ring
  // always takes once its oldest entries have moved out
  static constexpr unsigned kPop = kC >= 128u ? (unsigned)CC_CHUNK : kC / 2u;
  unsigned long long X[W * kC];
  unsigned long long E[W * kC];
  unsigned long long S[ENUM ? W * kC : 1];
  unsigned long long MG[kC];
  // the cached graph's rows (one- and two-word bitsets; four-word rows,
  // 8 KiB a graph, are read from device memory)
  static constexpr bool kRows = BATCH && W <= 2;
  unsigned long long rows[kRows ? CC_ROWS(W) * W : 1];
  unsigned long long hc[BATCH ? CC_ROWS(W) + 2 : 1];  // that graph's histogram, this
                                                      // wavefront's share not yet added
};

// A frame in registers (one per lane).
template <int W>
struct Frame {
  Bits<W> X, E, S;
  unsigned int m, gid;
};

template <int W, bool ENUM, bool BATCH>
__global__ __launch_bounds__(CC_BLOCK) void k_dfs(GraphDev g, CcCtl *ctl, Frontier f0,
                                                  Frontier f1, DfsWork wk,
                                                  OutDev out, unsigned long long *hist_out,
                                                  int hist_stride, int count_front,
                                                  unsigned long long idle_timeout, BatchDev bt) {
  using WL = DfsWaveLds<W, ENUM, BATCH>;
  constexpr unsigned C = WL::kC;
  __shared__ WL sW[CC_BLOCK / CC_WAVE];
  constexpr unsigned POP = WL::kPop;
  // rows in LDS up to 256 vertices, in device memory beyond
  __shared__ unsigned long long sN[BATCH || CC_BIG(W) ? 1 : CC_ROWS(W) * W];
  __shared__ unsigned long long sNo[ENUM && !CC_BIG(W) ? CC_ROWS(W) * W : 1];
  __shared__ int sPerm[BATCH ? 1 : CC_ROWS(W)];
  __shared__ unsigned long long sHist[BATCH ? 1 : CC_SLOTS(W)];
  __shared__ unsigned long long sFront[BATCH ? 1 : CC_SLOTS(W)];
  __shared__ long long sCb[ENUM ? CC_SLOTS(W) : 1];
  __shared__ long long sVb[ENUM ? CC_SLOTS(W) : 1];
  __shared__ unsigned long long sPre[CC_SHARDS + 1];
  if (!BATCH && ld_relaxed(&ctl->mode) == 0) return;
  const int L = BATCH ? 3 : ctl->switch_level;
  const int skipbits = BATCH ? 0 : ctl->skip;
  const Frontier roots = (!BATCH && ctl->root_buf) ? f1 : f0;
  const int n = g.n;
  const int tid = threadIdx.x;
  const int lane = lane_id();
  // the wavefront's index in the block, as a scalar (uniform) value: the
  // stack bookkeeping below then stays in scalar registers
  const int wib = __builtin_amdgcn_readfirstlane(tid / CC_WAVE);
  WL &Q = sW[wib];
  if (!BATCH && tid < CC_WAVE) {
    const unsigned long long c = ld_relaxed(&ctl->count_sh[lane][L]);
    shard_prefix(c <= roots.cap_s ? c : roots.cap_s, sPre);
  }
  if (!BATCH) {
    if (!CC_BIG(W))
      for (int i = tid; i < n * W; i += CC_BLOCK) sN[i] = g.adj[i];
    for (int i = tid; i < n; i += CC_BLOCK) sPerm[i] = g.perm[i];
    for (int i = tid; i < CC_SLOTS(W); i += CC_BLOCK) sHist[i] = 0ull;
  }
  if (!BATCH)
    for (int i = tid; i < CC_SLOTS(W); i += CC_BLOCK) sFront[i] = 0ull;
  const unsigned long long *const Nr = CC_BIG(W) ? g.adj : sN;
  const unsigned long long *const Nor = CC_BIG(W) ? g.adj_orig : sNo;
  if (ENUM) {
    if (!CC_BIG(W))
      for (int i = tid; i < n * W; i += CC_BLOCK) sNo[i] = g.adj_orig[i];
    for (int i = tid; i < CC_SLOTS(W); i += CC_BLOCK) {
      sCb[i] = (long long)ctl->len_cbase[i];
      sVb[i] = (long long)ctl->len_vbase[i];
    }
  }
  __syncthreads();
  const unsigned long long nroots = BATCH ? bt.r1 - bt.r0 : sPre[CC_SHARDS];
  // output index of the first cycle this kernel finds (the lengths above
  // bfs_max_len), for the staging of out.dstage
  const long long dfs_c0 = ENUM ? sCb[min(ctl->bfs_max_len + 1, CC_SLOTS(W) - 1)] : 0;

  const int wid = blockIdx.x * (CC_BLOCK / CC_WAVE) + wib;
  const int nwaves = gridDim.x * (CC_BLOCK / CC_WAVE);
  // device-memory stack of this wavefront: entries [bot, top) of cap (at
  // most 2^20, so 32-bit indices)
  const unsigned cap = (unsigned)wk.cap_w;
  unsigned long long *stX = wk.stackX + (unsigned long long)wid * W * cap;
  unsigned long long *stE = wk.stackE + (unsigned long long)wid * W * cap;
  unsigned long long *stS = ENUM ? wk.stackS + (unsigned long long)wid * W * cap : nullptr;
  unsigned int *stM = wk.stackM + (unsigned long long)wid * cap;
  unsigned int *stG = BATCH ? wk.stackG + (unsigned long long)wid * cap : nullptr;
  unsigned int *my_mail = wk.mail + (size_t)wid * CC_MAIL;
  const unsigned long long dmin = (unsigned long long)max(wk.donate_min, 2);
  const unsigned int root_meta = ((unsigned)L << 16) | (1u << 31);
  // Claim size: up to CC_ROOT_CLAIM paths, but small enough that every
  // wavefront gets several claims when the handed-over frontier is small.
  const unsigned long long claim =
      wk.claim > 0 ? (unsigned long long)wk.claim
                   : max((unsigned long long)CC_CHUNK,
                         min((unsigned long long)CC_ROOT_CLAIM,
                             nroots / ((unsigned long long)nwaves * 4) / CC_CHUNK * CC_CHUNK));
  const int check_every = max(wk.donate_check, 1);

  unsigned lb = 0, lt = 0;                 // LDS ring entries [lb, lt), positions mod C
  unsigned bot = 0, top = 0;               // device-memory entries, below the ring
  unsigned long long r_lo = 0, r_hi = 0;   // private range of handed-over paths
  // diagnostics, 32-bit in the loop (added to the control block before
  // any of them could pass 2^31, and at exit)
  unsigned batches = 0, donated = 0, lanes_used = 0, fills = 0, spills = 0, gatomics = 0;
  unsigned long long idle_clk = 0;
  unsigned long long rng = 0x9E3779B97F4A7C15ull * (unsigned long long)(wid + 1);
  int until_check = 1 + wid % check_every;
  unsigned mail_seen = 0u;                 // lane 0: the request word, as loaded at the last check
  int cur_g = -1, cur_vo = 0, cur_n = 0;   // BATCH: the graph whose rows (one- and two-word
                                           // bitsets) and histogram share are in LDS
  bool roots_done = false;
  const unsigned long long clk_start = wall_clock64();
  if (BATCH)
    for (int k = lane; k < CC_ROWS(W) + 2; k += CC_WAVE) Q.hc[k] = 0ull;
  if (lane == 0) atomicAdd(&ctl->busy, 1);

  auto ring_get = [&](unsigned i, Frame<W> &f) {
#pragma unroll
    for (int w = 0; w < W; ++w) {
      f.X.w[w] = Q.X[w * C + i];
      f.E.w[w] = Q.E[w * C + i];
    }
    if (ENUM) {
#pragma unroll
      for (int w = 0; w < W; ++w) f.S.w[w] = Q.S[w * C + i];
    }
    const unsigned long long mg = Q.MG[i];
    f.m = (unsigned)mg;
    f.gid = BATCH ? (unsigned)(mg >> 32) : 0u;
  };
  auto ring_put = [&](unsigned i, const Frame<W> &f) {
#pragma unroll
    for (int w = 0; w < W; ++w) {
      Q.X[w * C + i] = f.X.w[w];
      Q.E[w * C + i] = f.E.w[w];
    }
    if (ENUM) {
#pragma unroll
      for (int w = 0; w < W; ++w) Q.S[w * C + i] = f.S.w[w];
    }
    Q.MG[i] = (unsigned long long)f.m | (BATCH ? (unsigned long long)f.gid << 32 : 0ull);
  };
  auto dev_get = [&](unsigned d, Frame<W> &f) {
#pragma unroll
    for (int w = 0; w < W; ++w) {
      f.X.w[w] = stX[(size_t)w * cap + d];
      f.E.w[w] = stE[(size_t)w * cap + d];
    }
    if (ENUM) {
#pragma unroll
      for (int w = 0; w < W; ++w) f.S.w[w] = stS[(size_t)w * cap + d];
    }
    f.m = stM[d];
    if (BATCH) f.gid = stG[d];
  };
  auto dev_put = [&](unsigned d, const Frame<W> &f) {
#pragma unroll
    for (int w = 0; w < W; ++w) {
      stX[(size_t)w * cap + d] = f.X.w[w];
      stE[(size_t)w * cap + d] = f.E.w[w];
    }
    if (ENUM) {
#pragma unroll
      for (int w = 0; w < W; ++w) stS[(size_t)w * cap + d] = f.S.w[w];
    }
    stM[d] = f.m;
    if (BATCH) stG[d] = f.gid;
  };
  auto zero_frame = [&](Frame<W> &f) {
    f.X = bzero<W>();
    f.E = bzero<W>();
    f.S = bzero<W>();
    f.m = 0;
    f.gid = 0;
  };

  // BATCH: adds the wavefront's counts for graph cur_g to its histogram in
  // device memory and clears them.
  auto flush_hc = [&]() {
    if (BATCH && cur_g >= 0) {
      wave_lds_sync();
      for (int k = lane; k < cur_n + 2; k += CC_WAVE) {
        const unsigned long long h = Q.hc[k];
        if (h) {
          atomicAdd(&bt.hist[(size_t)cur_g * bt.hist_stride + k], h);
          Q.hc[k] = 0ull;
        }
      }
      wave_lds_sync();
    }
  };

  auto flush_diag = [&]() {
    if (lane == 0) {
      atomicAdd(&ctl->dfs_batches, (unsigned long long)batches);
      if (donated) atomicAdd(&ctl->donations, (unsigned long long)donated);
      atomicAdd(&ctl->dfs_lanes, (unsigned long long)lanes_used);
      if (fills) atomicAdd(&ctl->dfs_fills, (unsigned long long)fills);
      if (spills) atomicAdd(&ctl->dfs_spills, (unsigned long long)spills);
      if (gatomics) atomicAdd(&ctl->dfs_gatomics, (unsigned long long)gatomics);
    }
    batches = donated = lanes_used = fills = spills = gatomics = 0u;
  };

  // The frame of a handed-over path <q, vt> (a root): q's exclusion set and
  // ids, E = {vt}.  False for a padding slot of a batch.
  auto root_frame = [&](unsigned long long i, Frame<W> &f) -> bool {
    if (BATCH) {
      const unsigned long long e = bt.r0 + i;
      const unsigned gg = bt.rgid[e];
      if (gg == CC_NO_GRAPH) return false;
      const unsigned vv = bt.rvv[e];
#pragma unroll
      for (int w = 0; w < W; ++w) f.X.w[w] = bt.rX[w * bt.rcap + e];
      f.E = bsingle<W>((int)(vv >> 8));
      f.m = (vv & 0xffu) | root_meta;
      f.gid = gg;
    } else {
      const int s = shard_of(sPre, i);
      const unsigned long long e = (unsigned long long)s * roots.cap_s + (i - sPre[s]);
      const unsigned vv = vv_load<W>(roots, e);
      const int vt = vv_vt<W>(vv);
#pragma unroll
      for (int w = 0; w < W; ++w) f.X.w[w] = roots.X[w * roots.cap + e];
      f.E = bsingle<W>(vt);
      if (ENUM) {
        Bits<W> s0;
#pragma unroll
        for (int w = 0; w < W; ++w) s0.w[w] = roots.S[w * roots.cap + e];
        f.S = bandnot(s0, bsingle<W>(sPerm[vt < n ? vt : 0]));
      }
      f.m = (unsigned)vv_v1<W>(vv) | root_meta;
      f.gid = 0;
    }
    return true;
  };

  while (true) {
    // The stack bookkeeping is the same in every lane: pinned to scalar
    // registers, so the compiler branches on it without exec masks.
    lt = uni_u32(lt);
    lb = uni_u32(lb);
    top = uni_u32(top);
    bot = uni_u32(bot);
    r_lo = uni_u64(r_lo);
    r_hi = uni_u64(r_hi);
    until_check = (int)uni_u32((unsigned)until_check);
    if (BATCH) {
      cur_g = (int)uni_u32((unsigned)cur_g);
      cur_vo = (int)uni_u32((unsigned)cur_vo);
      cur_n = (int)uni_u32((unsigned)cur_n);
    }
    if (lt == lb) {
      // ---- the ring is empty: refill it from device memory, else from
      // the handed-over paths, else from another wavefront
      lb = lt = 0;
      if (top != bot) {
        // the newest entries of device memory, oldest first
        ++fills;
        const unsigned m = min(top - bot, C / 2u);
        for (unsigned c0 = 0; c0 < m; c0 += CC_CHUNK) {
          const unsigned j = c0 + (unsigned)lane;
          if (j < m) {
            Frame<W> f;
            zero_frame(f);
            dev_get(top - m + j, f);
            ring_put(j, f);
          }
        }
        lt = m;
        top -= m;
        if (top == bot) top = bot = 0;
      } else if (!roots_done || r_lo < r_hi) {
        if (r_lo >= r_hi) {
          unsigned long long c = ~0ull;
          if (lane == 0 && ld_relaxed(&ctl->root_cursor) < nroots)
            c = atomicAdd(&ctl->root_cursor, claim);
          c = lane_u64(c, 0);
          if (c < nroots) {
            r_lo = c;
            r_hi = min(c + claim, nroots);
          } else {
            roots_done = true;
          }
        }
        if (r_lo < r_hi) {
          const unsigned long long kk = min(r_hi - r_lo, (unsigned long long)CC_CHUNK);
          Frame<W> f;
          zero_frame(f);
          bool ok = false;
          if ((unsigned long long)lane < kk) ok = root_frame(r_lo + lane, f);
          const unsigned long long mk = wave_ballot(ok);
          if (ok) ring_put(lanes_below(mk), f);
          lt = (unsigned)__popcll(mk);
          r_lo += kk;
        }
      } else {
        // ---- idle: ask a busy wavefront for work, or leave when none is left
        if (lane == 0) {
          st_coh(&my_mail[3], 0u);
          atomicSub(&ctl->busy, 1);
        }
        int victim = -1;                 // wavefront our pending request went to
        unsigned long long t_req = 0;
        int outcome = 0;                 // 1: work delivered, 2: leave, 3: roots left, 4: gave up
        const unsigned long long t0 = wall_clock64();
        int backoff = 1;
        while (true) {
          int o = 0;
          if (lane == 0) {
            // decline whatever is asked of us while we have nothing
            const unsigned r = ld_coh(&my_mail[0]);
            if (r != 0u && r != CC_MAIL_CLOSED && atomicCAS(&my_mail[0], r, 0u) == r) {
              if (r - 1u < (unsigned)nwaves) st_coh(&wk.mail[(size_t)(r - 1) * CC_MAIL + 1], 2u);
              else dfs_corrupt(ctl, CC_DIAG_REQUESTER, r);
            }
            if (victim >= 0) {
              const unsigned resp = ld_coh(&my_mail[1]);
              if (resp == 1u) {
                o = 1;
              } else if (resp == 2u) {
                st_coh(&my_mail[1], 0u);
                victim = -1;
              } else if (wall_clock64() - t_req > 20000ull || ld_coh(&ctl->busy) == 0) {
                // withdraw; if the victim already took the request, keep waiting
                if (atomicCAS(&wk.mail[(size_t)victim * CC_MAIL], (unsigned)wid + 1u, 0u) ==
                    (unsigned)wid + 1u)
                  victim = -1;
              }
              // a taken request is always answered; if the answer never comes,
              // give up after the idle timeout and report the run incomplete
              if (o == 0 && victim >= 0 && wall_clock64() - t0 > idle_timeout) o = 5;
            }
            if (o == 0 && victim < 0) {
              if (!roots_done && ld_coh(&ctl->root_cursor) < nroots) o = 3;
              else if (ld_coh(&ctl->busy) == 0) o = 2;
              else if (wall_clock64() - t0 > idle_timeout) o = 4;
            }
          }
          // lane 0's decisions, as wavefront-uniform (scalar) values
          o = __builtin_amdgcn_readfirstlane(o);
          victim = __builtin_amdgcn_readfirstlane(victim);
          if (o != 0) {
            outcome = o;
            break;
          }
          if (victim < 0) {
            // pick the richest of 64 candidates by their published hints
            rng ^= rng << 13;
            rng ^= rng >> 7;
            rng ^= rng << 17;
            const int cand = (int)(((rng >> 16) + (unsigned long long)lane * 40503ull) %
                                   (unsigned long long)nwaves);
            unsigned hint = cand == wid ? 0u : ld_coh(&wk.mail[(size_t)cand * CC_MAIL + 3]);
            if (hint < dmin) hint = 0u;
            unsigned long long key = ((unsigned long long)hint << 32) | (unsigned)cand;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
              const unsigned long long other = __shfl_xor(key, off, CC_WAVE);
              key = other > key ? other : key;
            }
            key = lane_u64(key, 0);  // every lane holds the maximum
            if ((key >> 32) != 0ull) {
              const int v = (int)(key & 0xffffffffull);
              int ok = 0;
              if (lane == 0)
                ok = atomicCAS(&wk.mail[(size_t)v * CC_MAIL], 0u, (unsigned)wid + 1u) == 0u;
              ok = __builtin_amdgcn_readfirstlane(ok);
              if (ok) {
                victim = v;
                t_req = wall_clock64();
                backoff = 1;
                continue;
              }
            }
          }
          for (int z = 0; z < backoff; ++z) __builtin_amdgcn_s_sleep(16);
          backoff = min(backoff * 2, 32);
        }
        idle_clk += wall_clock64() - t0;
        if (outcome == 3) {
          if (lane == 0) atomicAdd(&ctl->busy, 1);
          continue;
        }
        if (outcome != 1) {
          if (outcome == 4 && lane == 0) atomicOr(&ctl->status, CC_DEV_IDLE_TIMEOUT);
          if (outcome == 5 && lane == 0) atomicOr(&ctl->status, CC_DEV_LOST);
          break;
        }
        // Work arrived in our inbox (the donor already counted us busy).  The
        // acquire pairs with the donor's release of the response word, so the
        // count and the paths below are the ones it wrote.
        acquire_agent();
        unsigned kk = 0;
        if (lane == 0) kk = ld_coh(&my_mail[2]);
        kk = (unsigned)__builtin_amdgcn_readlane((int)kk, 0);
        if (kk > (unsigned)CC_CHUNK) {
          if (lane == 0) dfs_corrupt(ctl, CC_DIAG_INBOX_COUNT, kk);
          kk = 0;
        }
        Frame<W> f;
        zero_frame(f);
        bool ok = (unsigned)lane < kk;
        if (ok) {
          const size_t ib = (size_t)wid * W * CC_CHUNK;
#pragma unroll
          for (int w = 0; w < W; ++w) {
            f.X.w[w] = ld_coh(&wk.inX[ib + w * CC_CHUNK + lane]);
            f.E.w[w] = ld_coh(&wk.inE[ib + w * CC_CHUNK + lane]);
          }
          if (ENUM) {
#pragma unroll
            for (int w = 0; w < W; ++w) f.S.w[w] = ld_coh(&wk.inS[ib + w * CC_CHUNK + lane]);
          }
          f.m = ld_coh(&wk.inM[(size_t)wid * CC_CHUNK + lane]);
          if (BATCH) {
            f.gid = ld_coh(&wk.inG[(size_t)wid * CC_CHUNK + lane]);
            ok = f.gid != CC_NO_GRAPH;  // a padding slot of the initial triplets
          }
        }
        wait_mem();
        if (lane == 0) st_coh(&my_mail[1], 0u);
        const unsigned long long mk = wave_ballot(ok);
        if (ok) ring_put(lanes_below(mk), f);
        lt = (unsigned)__popcll(mk);
      }
    }
    // ---- expand from the ring until it empties or a mailbox check is due
    while (lt != lb && until_check > 0) {
      --until_check;
      ++batches;
      // Keep a wavefront's worth of frames: top a short ring up from below
      // its bottom, with the newest entries of device memory, else with
      // paths of the private range of handed-over paths.  (Not in batches:
      // their rings are nearly always full, and a top-up would mix graphs
      // in one step.)
      if (!BATCH && lt - lb < POP) {
        if (top != bot) {
          ++fills;
          const unsigned m = min(top - bot, C / 2u - (lt - lb));
          for (unsigned c0 = 0; c0 < m; c0 += CC_CHUNK) {
            const unsigned j = c0 + (unsigned)lane;
            if (j < m) {
              Frame<W> f;
              zero_frame(f);
              dev_get(top - m + j, f);
              ring_put((lb - m + j) & (C - 1u), f);
            }
          }
          lb -= m;
          top -= m;
          if (top == bot) top = bot = 0;
          wave_lds_sync();
        } else if (r_lo < r_hi) {
          const unsigned long long kr =
              min(r_hi - r_lo, (unsigned long long)(POP - (lt - lb)));
          Frame<W> f;
          zero_frame(f);
          bool ok = false;
          if ((unsigned long long)lane < kr) ok = root_frame(r_lo + lane, f);
          const unsigned long long mk = wave_ballot(ok);
          const unsigned cnt = (unsigned)__popcll(mk);
          if (ok) ring_put((lb - cnt + lanes_below(mk)) & (C - 1u), f);
          lb -= cnt;
          r_lo += kr;
          wave_lds_sync();
        }
      }
      // Pop up to 64 frames from the top.  In the worst case every entry
      // left in the ring and both new frames of every popped one end up in
      // device memory: keep that within its capacity.
      unsigned kk = min(lt - lb, POP);
      while (kk > 1 && (top - bot) + (lt - lb) + kk > cap) kk >>= 1;
      const unsigned start = lt - kk;
      const bool in_step = (unsigned)lane < kk;
      bool valid = in_step;
      // every lane reads a ring slot; those past the popped ones hold stale
      // entries that nothing below uses (valid is false for them)
      Frame<W> f;
      ring_get((start + (unsigned)lane) & (C - 1u), f);
      lt = start;
      lanes_used += kk;
      // Consistency checks: every index below that comes from a frame
      // stays inside its graph; a frame that fails is reported and dropped.
      // (Each check is one wavefront-uniform branch, taken only on bad
      // state; predicates are combined without short-circuit branches.)
      int n_path = n;  // vertices of this frame's graph
      int vo = 0;
      // every frame of the step is of the cached graph cur_g (always, for one graph)
      bool in_cur = !BATCH;
      if (BATCH) {
        // usual case: every frame of the step is of the graph whose rows the
        // wavefront holds (lane 0 always has a frame)
        const unsigned g0 = uni_u32(f.gid);
        if ((int)g0 == cur_g && wave_ballot(in_step & (f.gid != g0)) == 0ull) {
          in_cur = true;
          vo = cur_vo;
          n_path = cur_n;
        } else {
          const bool bad_g = valid & (f.gid >= (unsigned)bt.n_graphs);
          if (wave_ballot(bad_g)) {
            if (bad_g) dfs_corrupt(ctl, CC_DIAG_GRAPH, f.gid);
            valid = valid & !bad_g;
          }
          f.gid = valid ? f.gid : 0u;
          const unsigned long long vm = wave_ballot(valid);
          if (vm) {
            const unsigned g1 = (unsigned)__builtin_amdgcn_readlane(
                (int)f.gid, (int)(__ffsll((long long)vm) - 1));
            if (wave_ballot(valid & (f.gid != g1)) == 0ull) {
              // one graph: its rows into LDS
              if ((int)g1 != cur_g) {
                flush_hc();
                cur_vo = bt.vtx_off[g1];
                cur_n = min(bt.vtx_off[g1 + 1] - cur_vo, CC_ROWS(W));
                if (cur_n < 0) cur_n = 0;
                if (WL::kRows)
                  for (int i = lane; i < cur_n * W; i += CC_WAVE)
                    Q.rows[i] = bt.adj[(size_t)cur_vo * W + i];
                cur_g = (int)g1;
              }
              in_cur = true;
              vo = cur_vo;
              n_path = cur_n;
            } else {
              vo = bt.vtx_off[f.gid];
              n_path = bt.vtx_off[f.gid + 1] - vo;
            }
          }
        }
      }
      // the path to expand: <q, v> for the lowest v of E (an empty E gives
      // some v, and the frame is rejected below)
      const bool has_e = bany(f.E);
      int v = bpop_lowest(f.E);
      {
        const int pv1 = f.m & 0xffffu, pt = (f.m >> 16) & 0x7ffu;
        const bool bad = valid & (!has_e | (pv1 >= n_path) | ((unsigned)v >= (unsigned)n_path) |
                                  (pt < 3) | (pt > n_path));
        if (wave_ballot(bad)) {
          if (bad)
            dfs_corrupt(ctl, CC_DIAG_PATH,
                        has_e && !CC_BIG(W) ? (f.m & 0xffff00ffu) | ((unsigned)(v & 0xff) << 8) : f.m);
          valid = valid & !bad;
        }
      }
      if (!valid) {
        f.m = 0;
        f.E = bzero<W>();
        v = 0;
      }
      const int v1 = f.m & 0xffffu;
      const int t = (f.m >> 16) & 0x7ffu;
      const bool root = (f.m >> 31) != 0;
      const bool count_path = valid && !(root && (skipbits & CC_SKIP_FRONT));
      const bool count_close = valid && !(root && (skipbits & CC_SKIP_CLOSE));
      Bits<W> nvt, nv1;
      if (BATCH && !(WL::kRows && in_cur)) {
        // rows from device memory (a step that mixes graphs, or four-word rows)
#pragma unroll
        for (int w = 0; w < W; ++w) {
          nvt.w[w] = bt.adj[(size_t)(vo + v) * W + w];
          nv1.w[w] = bt.adj[(size_t)(vo + v1) * W + w];
        }
      } else {
        nvt = row<W>(BATCH ? Q.rows : Nr, v);
        nv1 = row<W>(BATCH ? Q.rows : Nr, v1);
      }
      const Bits<W> cand = bandnot(nvt, f.X);
      Bits<W> clos = band(cand, nv1);
      Bits<W> ext = bandnot(cand, nv1);
      if (!valid) {
        clos = bzero<W>();
        ext = bzero<W>();
      }
      if (!BATCH && count_front && count_path) {
        // paths expanded, per length
        atomicAdd(&sFront[t], 1ull);
      }
      // the expanded path's own original ids (enumerate)
      const Bits<W> Sp = ENUM ? bor(f.S, bsingle<W>(sPerm[v])) : bzero<W>();
      if (BATCH && in_cur) {
        // every frame is of graph cur_g: each lane adds its closures to the
        // wavefront's LDS share of that graph's histogram
        const unsigned c = count_close ? (unsigned)bpop(clos) : 0u;
        if (c) atomicAdd(&Q.hc[t + 1], (unsigned long long)c);
      } else if (BATCH) {
        // frames of several graphs: one global add per distinct (graph,
        // length) among the lanes
        const unsigned c = count_close ? (unsigned)bpop(clos) : 0u;
        const unsigned key = (f.gid << 8) | (unsigned)(t + 1);
        unsigned long long act = wave_ballot(c != 0u);
        while (act) {
          const unsigned k0 =
              (unsigned)__builtin_amdgcn_readlane((int)key, (int)(__ffsll((long long)act) - 1));
          const unsigned long long same = act & wave_ballot(key == k0);
          const unsigned sum = wave_sum_u32_full((same >> lane) & 1ull ? c : 0u);
          if (lane == 0)
            atomicAdd(&bt.hist[(size_t)(k0 >> 8) * bt.hist_stride + (k0 & 0xffu)],
                      (unsigned long long)sum);
          ++gatomics;
          act &= ~same;
        }
      } else if (count_close) {
        const int c = bpop(clos);
        if (c) {
          if (hist_out) atomicAdd(&sHist[t + 1], (unsigned long long)c);
          if (ENUM) {
            const int k = t + 1;
            if (k >= out.kmin && k <= out.kmax) {
              const unsigned long long slot0 =
                  atomicAdd(&ctl->len_cursor[k], (unsigned long long)c);
              Bits<W> cl = clos;
              for (int j = 0; j < c; ++j) {
                const int w = bpop_lowest(cl);
                long long cyc = sCb[k] + (long long)(slot0 + j);
                long long pos = sVb[k] + (long long)(slot0 + j) * k;
                const long long si = cyc - dfs_c0;
                if (out.dstage && si >= 0 && si < out.dstage_cap) {
                  // staged; k_dfs_decode writes it with every lane busy
                  const Bits<W> Cy = bor(Sp, bsingle<W>(sPerm[w]));
#pragma unroll
                  for (int q = 0; q < W; ++q) out.dstage[q * out.dstage_cap + si] = Cy.w[q];
                } else if (out_slot(out, k, cyc, pos)) {
                  write_cycle<W>(Nor, bor(Sp, bsingle<W>(sPerm[w])), k, out.verts + pos);
                  out.offs[cyc] = pos;
                }
              }
            }
          }
        }
      }
      // A path never has more than n vertices (each extension adds a vertex
      // outside the path, and the path is inside X); anything longer would
      // mean corrupted state, so it is dropped and reported instead of
      // looping.
      {
        const bool too_long = t >= n_path && bany(ext);
        if (wave_ballot(too_long)) {
          if (lane == 0) atomicOr(&ctl->status, CC_DEV_STACK_FULL);
          if (too_long) ext = bzero<W>();
        }
      }
      // ---- push: what is left of E, then the new frame of the extensions
      // on top of it (at most 2 POP <= C entries, so the ring always takes
      // them once its oldest entries have moved out)
      const bool push_rem = valid && bany(f.E);
      const bool push_ext = valid && bany(ext);
      const unsigned long long m_rem = wave_ballot(push_rem);
      const unsigned long long m_ext = wave_ballot(push_ext);
      const unsigned n_rem = (unsigned)__popcll(m_rem);
      const unsigned tot = n_rem + (unsigned)__popcll(m_ext);
      if (tot) {
        const unsigned used = lt - lb;
        if (used + tot > C) {
          // Move the ring's oldest entries to device memory, whole
          // wavefront chunks at a time.
          const unsigned spill =
              min(used, (used + tot - C + (unsigned)CC_CHUNK - 1u) / CC_CHUNK * CC_CHUNK);
          if (top + spill > cap && bot > 0) {
            // Slide the device-memory part down to index 0, 64 entries at
            // a time: a chunk's loads all complete before its stores, and
            // later chunks only read above what earlier chunks wrote.
            const unsigned live = top - bot;
            for (unsigned c0 = 0; c0 < live; c0 += CC_CHUNK) {
              const unsigned i = c0 + (unsigned)lane;
              if (i < live) {
                Frame<W> d;
                zero_frame(d);
                dev_get(bot + i, d);
                dev_put(i, d);
              }
            }
            top = live;
            bot = 0;
          }
          if (top + spill > cap) {
            // cannot happen with the pop size above; reported, not looped on
            if (lane == 0) atomicOr(&ctl->status, CC_DEV_STACK_FULL);
            lb += spill;
          } else {
            for (unsigned c0 = 0; c0 < spill; c0 += CC_CHUNK) {
              const unsigned j = c0 + (unsigned)lane;
              if (j < spill) {
                Frame<W> d;
                zero_frame(d);
                ring_get((lb + j) & (C - 1u), d);
                dev_put(top + j, d);
              }
            }
            top += spill;
            lb += spill;
            spills += spill;
          }
          wave_lds_sync();  // the ring slots just read may be written below
        }
        if (push_rem) ring_put((lt + lanes_below(m_rem)) & (C - 1u), f);
        if (push_ext) {
          Frame<W> e;
#pragma unroll
          for (int w = 0; w < W; ++w) e.X.w[w] = f.X.w[w] | nvt.w[w];
          e.E = ext;
          e.S = Sp;
          e.m = (unsigned)v1 | ((unsigned)(t + 1) << 16);
          e.gid = f.gid;
          ring_put((lt + n_rem + lanes_below(m_ext)) & (C - 1u), e);
        }
        lt += tot;
      }
    }

    // ---- every few steps: publish what we could give, answer a request
    if (until_check <= 0) {
      until_check = check_every;
      if ((batches | lanes_used | spills) >= (1u << 31)) flush_diag();
      const unsigned long long range_left = r_hi - r_lo, dev_left = top - bot;
      const unsigned long long stack_left = dev_left + (unsigned long long)(lt - lb);
      const unsigned long long left = range_left + stack_left;
      // The request word was loaded at the previous check, so a check never
      // waits for memory unless there is a request to take.
      unsigned req = 0;
      const unsigned r = (unsigned)__builtin_amdgcn_readlane((int)mail_seen, 0);
      if (lane == 0) {
        st_coh(&my_mail[3], (unsigned)min(left, 0x7fffffffull));
        if (r != 0u && r != CC_MAIL_CLOSED && atomicCAS(&my_mail[0], r, 0u) == r) req = r;
        mail_seen = ld_coh(&my_mail[0]);
      }
      req = (unsigned)__builtin_amdgcn_readlane((int)req, 0);
      if (req != 0u && req - 1u >= (unsigned)nwaves) {
        if (lane == 0) dfs_corrupt(ctl, CC_DIAG_REQUESTER, req);
        req = 0u;
      }
      if (req != 0u) {
        const int q = (int)req - 1;
        unsigned int *q_mail = wk.mail + (size_t)q * CC_MAIL;
        const bool from_range = range_left >= dmin;
        if (from_range || stack_left >= dmin) {
          const unsigned give = (unsigned)min(
              (from_range ? range_left : stack_left) / 2, (unsigned long long)CC_CHUNK);
          const bool mine = (unsigned)lane < give;
          // the oldest stack entries: device memory first; when it holds
          // fewer than `give`, the ring holds at least that many
          const bool from_dev = dev_left >= give;
          Frame<W> d;
          zero_frame(d);
          if (from_range) {
            // padding slots travel as frames the recipient drops
            if (mine && !root_frame(r_hi - give + lane, d)) d.gid = CC_NO_GRAPH;
            r_hi -= give;
          } else if (from_dev) {
            if (mine) dev_get(bot + (unsigned)lane, d);
            bot += give;
            if (top == bot) top = bot = 0;
          } else {
            if (mine) ring_get((lb + (unsigned)lane) & (C - 1u), d);
            lb += give;
          }
          if (mine) {
            const size_t ib = (size_t)q * W * CC_CHUNK;
#pragma unroll
            for (int w = 0; w < W; ++w) {
              st_coh(&wk.inX[ib + w * CC_CHUNK + lane], d.X.w[w]);
              st_coh(&wk.inE[ib + w * CC_CHUNK + lane], d.E.w[w]);
            }
            if (ENUM) {
#pragma unroll
              for (int w = 0; w < W; ++w) st_coh(&wk.inS[ib + w * CC_CHUNK + lane], d.S.w[w]);
            }
            st_coh(&wk.inM[(size_t)q * CC_CHUNK + lane], d.m);
            if (BATCH) st_coh(&wk.inG[(size_t)q * CC_CHUNK + lane], d.gid);
          }
          if (lane == 0) {
            st_coh(&q_mail[2], give);
            atomicAdd(&ctl->busy, 1);  // the recipient holds work from now on
          }
          // every lane's inbox stores are visible before lane 0 publishes them
          release_agent();
          if (lane == 0) st_coh(&q_mail[1], 1u);
          ++donated;
        } else if (lane == 0) {
          st_coh(&q_mail[1], 2u);
        }
      }
    }
  }

  flush_hc();
  // Close the mailbox; decline a request that arrived meanwhile.
  if (lane == 0) {
    const unsigned r = atomicExch(&my_mail[0], CC_MAIL_CLOSED);
    if (r != 0u && r != CC_MAIL_CLOSED) {
      if (r - 1u < (unsigned)nwaves) st_coh(&wk.mail[(size_t)(r - 1) * CC_MAIL + 1], 2u);
      else dfs_corrupt(ctl, CC_DIAG_REQUESTER, r);
    }
    atomicAdd(&ctl->dfs_idle_clk, idle_clk);
    atomicAdd(&ctl->dfs_wave_clk, wall_clock64() - clk_start);
  }
  flush_diag();
  __syncthreads();
  unsigned long long *hdst = hist_out ? hist_out + (size_t)(blockIdx.x % CC_SHARDS) * hist_stride
                                      : nullptr;
  for (int i = tid; i < CC_SLOTS(W); i += CC_BLOCK) {
    if (!BATCH && hdst && sHist[i]) atomicAdd(&hdst[i], sHist[i]);
    if (!BATCH && count_front && sFront[i]) atomicAdd(&ctl->front[i], sFront[i]);
  }
}


// Resets the depth-first coordination state: every mailbox of the
// workspace, the claim cursor and the busy count, unconditionally (the
// workspace has memory of its own, so nothing else ever lives there); for
// the writing pass of enumerate mode it also computes where each cycle
// length starts in the output.
// The cycles the depth-first kernel staged (out.dstage), decoded the way a
// step decodes its staged cycles: per length above bfs_max_len, runs of
// cycles per wavefront, each lane walking one cycle into LDS, then the
// run's vertex range written by consecutive lanes.  Returns at once when
// the levels finished without a hand-over.
template <int W>
__global__ __launch_bounds__(CC_BLOCK) void k_dfs_decode(GraphDev g, const CcCtl *ctl,
                                                         OutDev out) {
  constexpr int NWB = CC_BLOCK / CC_WAVE;
  __shared__ unsigned long long sNo[CC_BIG(W) ? 1 : CC_ROWS(W) * W];
  __shared__ int sDec[NWB][CC_DEC_WORDS];
  __shared__ unsigned long long sPre[CC_SHARDS + 1];
  if (ctl->mode == 0 || !out.dstage) return;
  const int n = g.n, tid = threadIdx.x, wave = tid / CC_WAVE;
  if (!CC_BIG(W))
    for (int i = tid; i < n * W; i += CC_BLOCK) sNo[i] = g.adj_orig[i];
  const unsigned long long *const No = CC_BIG(W) ? g.adj_orig : sNo;
  const int L = ctl->bfs_max_len;
  const long long c0 = (long long)ctl->len_cbase[L + 1];
  const unsigned long long gw = (unsigned long long)blockIdx.x * NWB + wave;
  const unsigned long long nwg = (unsigned long long)gridDim.x * NWB;
  for (int k = L + 1; k <= n; ++k) {
    const long long cb = (long long)ctl->len_cbase[k];
    const long long si0 = cb - c0;
    // the staged ones (the rest went straight to the output)
    const long long h = min((long long)ctl->len_cbase[k + 1] - cb,
                            max(0ll, out.dstage_cap - si0));
    if (h <= 0) continue;
    // one shard holding all h cycles
    __syncthreads();  // the previous length's readers of sPre are done
    if (tid <= CC_SHARDS) sPre[tid] = tid == 0 ? 0ull : (unsigned long long)h;
    __syncthreads();
    Stage st;
    st.C = out.dstage + si0;
    st.cap = (unsigned long long)out.dstage_cap;
    st.cap_s = (unsigned long long)out.dstage_cap;
    decode_run<W, true>(No, sDec[wave], st, sPre, (unsigned long long)h, k, cb,
                        (long long)ctl->len_vbase[k], out, gw, nwg);
  }
}

__global__ void k_dfs_prepare(CcCtl *ctl, DfsWork wk, int n, int enum_bases) {
  __shared__ unsigned long long sTot[CC_HSLOTS];
  // the four words in use of every mailbox line (request, response, count,
  // hint); the rest of the line is padding
  const size_t words = (size_t)wk.nwaves * 4;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < words;
       i += (size_t)gridDim.x * blockDim.x)
    wk.mail[(i >> 2) * CC_MAIL + (i & 3)] = 0u;
  if (blockIdx.x != 0) return;
  if (enum_bases) length_totals(ctl, n, true, sTot);
  if (threadIdx.x == 0) {
    ctl->root_cursor = 0;
    ctl->busy = 0;
    if (enum_bases) {
      long long cb = 0, vb = 0;
      for (int k = 0; k < CC_HSLOTS; ++k) {
        ctl->len_cbase[k] = (unsigned long long)cb;
        ctl->len_vbase[k] = (unsigned long long)vb;
        ctl->len_cursor[k] = 0;
        cb += (long long)sTot[k];
        vb += (long long)sTot[k] * k;
      }
    }
  }
}

// ------------------------------------------------------------ sorted output
// Sorts the enumerated cycles of each length into ascending lexicographic
// order of their canonical vertex lists (the cycles of one length are
// fixed-size records of k original ids at a fixed stride, so the offsets do
// not change).  One block per length, all lengths in one launch: a stable
// LSD radix sort of the record indices with one byte digit per position (two,
// low byte first, when ids reach 256), last position first, then one gather
// of the records.
//   verts   the output (window relative); tmp has room for its vertex ids;
//   ia, ib  index scratch of at least the window's cycle count each.
// The lengths' places in the output come from the final histogram.  If the
// output did not fit the caller's buffers nothing is touched.
constexpr int kSortThreads = 1024;
__global__ __launch_bounds__(kSortThreads) void k_sort_cycles(const CcCtl *ctl, OutDev out,
                                                              int n, int *tmp, unsigned *ia0,
                                                              unsigned *ib0) {
  constexpr int NW = kSortThreads / CC_WAVE;
  __shared__ unsigned long long sh[4];
  __shared__ unsigned base[256];
  __shared__ unsigned wcnt[NW][257];
  const int k = blockIdx.x;
  const int tid = threadIdx.x, lane = lane_id(), wv = tid / CC_WAVE;
  if (k < 3 || k > n || k < out.kmin || k > out.kmax) return;
  if (tid == 0) {
    unsigned long long cb = 0, vb = 0, tc = 0, tv = 0;
    for (int j = 0; j <= n && j < CC_HSLOTS; ++j) {
      if (j < out.kmin || j > out.kmax) continue;
      const unsigned long long h = ctl->hist[j];
      if (j < k) {
        cb += h;
        vb += h * (unsigned long long)j;
      }
      tc += h;
      tv += h * (unsigned long long)j;
    }
    const bool fits = tc <= (unsigned long long)out.cyc_cap && tv <= (unsigned long long)out.verts_cap;
    sh[0] = cb;
    sh[1] = vb;
    sh[2] = fits ? ctl->hist[k] : 0ull;
  }
  __syncthreads();
  const unsigned long long cb = sh[0], vb = sh[1], cnt = sh[2];
  if (cnt < 2) return;
  const int *src = out.verts + vb;
  unsigned *ia = ia0 + cb, *ib = ib0 + cb;
  for (unsigned long long i = tid; i < cnt; i += kSortThreads) ia[i] = (unsigned)i;
  __syncthreads();
  const int nd = n > 256 ? 2 : 1;  // byte digits per position
  for (int p = k * nd - 1; p >= 0; --p) {
    const int pos = p / nd, sh = (nd - 1 - p % nd) * 8;
    // digit counts of the whole length, then where each digit starts
    for (int d = tid; d < 256; d += kSortThreads) base[d] = 0u;
    __syncthreads();
    for (unsigned long long i = tid; i < cnt; i += kSortThreads)
      atomicAdd(&base[(src[(unsigned long long)ia[i] * k + pos] >> sh) & 0xff], 1u);
    __syncthreads();
    if (tid < CC_WAVE) {
      // exclusive scan of 256 counts: four per lane, then across lanes
      unsigned c[4], s = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        c[q] = base[tid * 4 + q];
        s += c[q];
      }
      unsigned incl = s;
#pragma unroll
      for (int o = 1; o < CC_WAVE; o <<= 1) {
        const unsigned y = __shfl_up(incl, o, CC_WAVE);
        if (lane >= o) incl += y;
      }
      unsigned run = incl - s;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        base[tid * 4 + q] = run;
        run += c[q];
      }
    }
    __syncthreads();
    // stable scatter, 1024 records at a time in index order: a record's
    // place is its digit's start, plus the records of that digit in earlier
    // wavefronts of the chunk, plus those at lower lanes of its wavefront
    for (unsigned long long c0 = 0; c0 < cnt; c0 += kSortThreads) {
      const unsigned long long i = c0 + tid;
      const bool has = i < cnt;
      const unsigned d =
          has ? (unsigned)((src[(unsigned long long)ia[i] * k + pos] >> sh) & 0xff) : 256u;
      unsigned long long same = ~0ull;
#pragma unroll
      for (int b = 0; b < 9; ++b) {
        const unsigned long long mb = wave_ballot((d >> b) & 1u);
        same &= ((d >> b) & 1u) ? mb : ~mb;
      }
      const unsigned rank = lanes_below(same);
      for (int e = tid; e < NW * 257; e += kSortThreads) (&wcnt[0][0])[e] = 0u;
      __syncthreads();
      if (rank == 0) wcnt[wv][d] = (unsigned)__popcll(same);
      __syncthreads();
      if (has) {
        unsigned off = base[d] + rank;
        for (int w = 0; w < wv; ++w) off += wcnt[w][d];
        ib[off] = ia[i];
      }
      __syncthreads();
      for (int e = tid; e < 256; e += kSortThreads) {
        unsigned add = 0;
        for (int w = 0; w < NW; ++w) add += wcnt[w][e];
        base[e] += add;
      }
      __syncthreads();
    }
    unsigned *x = ia;
    ia = ib;
    ib = x;
  }
  // records in sorted order into tmp, then back over the length's range
  int *dst = tmp + vb;
  const unsigned long long nv = cnt * (unsigned long long)k;
  for (unsigned long long e = tid; e < nv; e += kSortThreads) {
    const unsigned long long r = e / (unsigned)k, j = e - r * (unsigned)k;
    dst[e] = src[(unsigned long long)ia[r] * k + j];
  }
  __syncthreads();
  int *o = out.verts + vb;
  for (unsigned long long e = tid; e < nv; e += kSortThreads) o[e] = dst[e];
}

// ------------------------------------------- the output grouped by root
// A finished enumeration, regrouped so that the cycles of each stage-one
// root are contiguous (roots in the order the root-range calls number
// them): every cycle gets its root's number, a stable radix sort orders the
// cycle indices by it, a scan gives the new offsets and a gather moves the
// vertex ids.  A range of roots is then one contiguous page.

// root_base[l]: the number of the first root whose u has label l (roots by
// u's original id, then x's, then y's).  One thread: n <= 1024 steps.
template <int W>
__global__ void k_root_base(GraphDev g, const int *label, long long *root_base) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  long long acc = 0;
  for (int v = 0; v < g.n; ++v) {
    const int l = label[v];
    if (l < 0 || l >= g.n) continue;
    const long long dp = bpop(bandnot(row<W>(g.adj, l), low_through<W>(l)));
    root_base[l] = acc;
    acc += dp * (dp - 1) / 2;
  }
}

// The root of each cycle: u is its vertex of smallest label, x and y the
// neighbours of u on the cycle, l(x) < l(y); its number follows the
// stage-one numbering (u's first root, plus the roots of u's higher
// neighbours x' before x by original id, plus y's rank among x's partners
// by original id).  key[i] = that number, idx[i] = i.
//
// Each wavefront takes runs of up to 64 consecutive cycles: their ids are
// copied into its LDS buffer by coalesced loads, then each lane walks one
// cycle there, starting at a lane-dependent position so that the lanes'
// reads of one round fall in different banks.
constexpr int kKeyBuf = CC_MAXN;  // ids per wavefront buffer (a cycle has at most n)
template <int W>
__global__ __launch_bounds__(CC_BLOCK) void k_cycle_root_keys(GraphDev g, const int *label,
                                                              const long long *root_base,
                                                              const int *verts,
                                                              const long long *offs,
                                                              long long nc, long long R,
                                                              unsigned *key, unsigned *idx) {
  constexpr int NW = CC_BLOCK / CC_WAVE;
  // rows in LDS up to 256 vertices, in device memory beyond
  __shared__ unsigned long long sN[CC_BIG(W) ? 1 : CC_ROWS(W) * W];
  __shared__ int sLab[CC_ROWS(W)], sPerm[CC_ROWS(W)];
  __shared__ long long sBase[CC_ROWS(W)];
  __shared__ int sBuf[NW][kKeyBuf];
  const int n = g.n;
  if (!CC_BIG(W))
    for (int i = threadIdx.x; i < n * W; i += CC_BLOCK) sN[i] = g.adj[i];
  const unsigned long long *const Nk = CC_BIG(W) ? g.adj : sN;
  for (int i = threadIdx.x; i < n; i += CC_BLOCK) {
    sLab[i] = label[i];
    sPerm[i] = g.perm[i];
    sBase[i] = root_base[i];
  }
  __syncthreads();
  const int lane = lane_id(), wave = threadIdx.x / CC_WAVE;
  int *buf = sBuf[wave];
  const long long nwg = (long long)gridDim.x * NW;
  // each wavefront owns blocks of 64 consecutive cycles, walked in runs
  // whose ids fit its buffer
  for (long long B = ((long long)blockIdx.x * NW + wave) * CC_WAVE; B < nc; B += nwg * CC_WAVE) {
    const long long bend = min(B + CC_WAVE, nc);
    long long j0 = B;
    while (j0 < bend) {
      const long long j = j0 + lane;
      const bool in = j < bend;
      const long long b = in ? offs[j] : 0, e = in ? offs[j + 1] : 0;
      const long long base = (long long)uni_u64((unsigned long long)offs[j0]);
      // the run: the cycles from j0 whose ids fit the buffer (at least one,
      // a cycle having at most n ids)
      const int nb = max(1, (int)__popcll(wave_ballot(in && e - base <= kKeyBuf)));
      const long long end = (long long)lane_u64((unsigned long long)e, nb - 1);
      {
        // sixteen loads in flight per round
        const int m = (int)(end - base);
        for (int q0 = 0; q0 < m; q0 += 16 * CC_WAVE) {
          int v[16];
#pragma unroll
          for (int u = 0; u < 16; ++u) {
            const int q = q0 + u * CC_WAVE + lane;
            v[u] = q < m ? verts[base + q] : 0;
          }
#pragma unroll
          for (int u = 0; u < 16; ++u) {
            const int q = q0 + u * CC_WAVE + lane;
            if (q < m) buf[q] = v[u];
          }
        }
      }
      wave_lds_sync();
      if (lane < nb) {
        const int s0 = (int)(b - base), k = (int)(e - b);
        int p = 0, lu = n;
        int q = k > 0 ? lane % k : 0;
        for (int t = 0; t < k; ++t) {
          const int v = buf[s0 + q];
          const int l = (v >= 0 && v < n) ? sLab[v] : n;
          if (l < lu) {
            lu = l;
            p = q;
          }
          if (++q == k) q = 0;
        }
        long long r = R;  // a malformed cycle (none in a finished run) sorts last
        if (k >= 3 && lu < n) {
          const int va = buf[s0 + (p + k - 1) % k], vc = buf[s0 + (p + 1) % k];
          const int la = (va >= 0 && va < n) ? sLab[va] : n;
          const int lc = (vc >= 0 && vc < n) ? sLab[vc] : n;
          if (la < n && lc < n && la != lc) {
            const int lx = min(la, lc), ly = max(la, lc);
            const Bits<W> up = bandnot(row<W>(Nk, lu), low_through<W>(lu));
            long long ix = sBase[lu];
            Bits<W> it = up;
            while (bany(it)) {
              const int xp = bpop_lowest(it);
              if (sPerm[xp] < sPerm[lx]) ix += bpop(bandnot(up, low_through<W>(xp)));
            }
            it = bandnot(up, low_through<W>(lx));
            while (bany(it)) {
              const int yp = bpop_lowest(it);
              ix += sPerm[yp] < sPerm[ly] ? 1 : 0;
            }
            r = ix < R ? ix : R;
          }
        }
        key[j] = (unsigned)r;
        idx[j] = (unsigned)j;
      }
      wave_lds_sync();  // the next run overwrites the buffer
      j0 += nb;
    }
  }
}

// Stable LSD radix sort of (key, idx) by 8-bit digits, multi-block: each
// block owns a tile of kRsTile items.  Pass: per-block digit counts
// (digit-major table, so that its exclusive scan gives every (digit, block)
// its first output slot), then a scatter that ranks the items of a tile in
// index order: per wavefront by matching digits with ballots, across the
// wavefronts of a round and across rounds by per-digit running counts.
constexpr int kRsThreads = 256;
constexpr int kRsIpt = 8;
constexpr int kRsTile = kRsThreads * kRsIpt;

__global__ __launch_bounds__(kRsThreads) void k_rs_count(const unsigned *key, long long n,
                                                         int shift, long long *table, int nb) {
  __shared__ unsigned c[256];
  c[threadIdx.x] = 0u;
  __syncthreads();
  const long long t0 = (long long)blockIdx.x * kRsTile;
  for (int r = 0; r < kRsIpt; ++r) {
    const long long i = t0 + (long long)r * kRsThreads + threadIdx.x;
    if (i < n) atomicAdd(&c[(key[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  table[(long long)threadIdx.x * nb + blockIdx.x] = (long long)c[threadIdx.x];
}

__global__ __launch_bounds__(kRsThreads) void k_rs_scatter(const unsigned *kin, const unsigned *vin,
                                                           unsigned *kout, unsigned *vout,
                                                           long long n, int shift,
                                                           const long long *table, int nb) {
  constexpr int NW = kRsThreads / CC_WAVE;
  __shared__ long long base[256];
  __shared__ long long wc[NW][256];
  const int tid = threadIdx.x, lane = lane_id(), wave = tid / CC_WAVE;
  base[tid] = table[(long long)tid * nb + blockIdx.x];
  const long long t0 = (long long)blockIdx.x * kRsTile;
  const unsigned long long below = (1ull << lane) - 1ull;
  for (int r = 0; r < kRsIpt; ++r) {
    for (int w = 0; w < NW; ++w) wc[w][tid] = 0;
    __syncthreads();
    const long long i = t0 + (long long)r * kRsThreads + tid;
    const bool valid = i < n;
    const unsigned kv = valid ? kin[i] : 0u;
    const unsigned vv = valid ? vin[i] : 0u;
    const unsigned d = (kv >> shift) & 255u;
    // lanes of this wavefront with the same digit
    unsigned long long m = wave_ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const bool on = (d >> bit) & 1u;
      const unsigned long long mb = wave_ballot(on);
      m &= on ? mb : ~mb;
    }
    const int rank = __popcll(m & below);
    if (valid && rank == 0) wc[wave][d] = __popcll(m);
    __syncthreads();
    {
      // digit tid: running counts across the wavefronts of this round
      long long run = base[tid];
      for (int w = 0; w < NW; ++w) {
        const long long c = wc[w][tid];
        wc[w][tid] = run;
        run += c;
      }
      base[tid] = run;
    }
    __syncthreads();
    if (valid) {
      const long long pos = wc[wave][d] + rank;
      kout[pos] = kv;
      vout[pos] = vv;
    }
    __syncthreads();
  }
}

// Exclusive scan of int64 values in place, by tiles of kScanTile: each tile
// is scanned by one block (its total to totals[block]); the host scans the
// totals the same way and adds them back.
constexpr int kScanThreads = 1024;
constexpr int kScanIpt = 4;
constexpr int kScanTile = kScanThreads * kScanIpt;

__global__ __launch_bounds__(kScanThreads) void k_scan_tile(long long *x, long long n,
                                                            long long *totals) {
  constexpr int NW = kScanThreads / CC_WAVE;
  __shared__ long long sw[NW];
  const int tid = threadIdx.x, lane = lane_id(), wave = tid / CC_WAVE;
  const long long b = (long long)blockIdx.x * kScanTile + (long long)tid * kScanIpt;
  long long v[kScanIpt];
  long long s = 0;
#pragma unroll
  for (int j = 0; j < kScanIpt; ++j) {
    v[j] = b + j < n ? x[b + j] : 0;
    s += v[j];
  }
  // inclusive scan over the wavefront, then over the wavefronts' totals
  long long inc = s;
#pragma unroll
  for (int o = 1; o < CC_WAVE; o <<= 1) {
    const long long t = __shfl_up(inc, o, CC_WAVE);
    if (lane >= o) inc += t;
  }
  if (lane == CC_WAVE - 1) sw[wave] = inc;
  __syncthreads();
  if (tid == 0) {
    long long run = 0;
    for (int w = 0; w < NW; ++w) {
      const long long t = sw[w];
      sw[w] = run;
      run += t;
    }
    if (totals) totals[blockIdx.x] = run;
  }
  __syncthreads();
  long long run = sw[wave] + inc - s;
#pragma unroll
  for (int j = 0; j < kScanIpt; ++j) {
    if (b + j < n) x[b + j] = run;
    run += v[j];
  }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_add(long long *x, long long n,
                                                           const long long *add) {
  const long long b = (long long)blockIdx.x * kScanTile + (long long)threadIdx.x * kScanIpt;
  const long long a = add[blockIdx.x];
#pragma unroll
  for (int j = 0; j < kScanIpt; ++j)
    if (b + j < n) x[b + j] += a;
}

// New lengths in sorted order: len[j] = length of cycle idx[j]; the slot
// after the last holds 0 (so that the exclusive scan of nc + 1 entries ends
// with the total).
__global__ void k_sorted_lengths(const unsigned *idx, const long long *offs, long long nc,
                                 long long *len) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x; j <= nc; j += stride)
    len[j] = j < nc ? offs[(long long)idx[j] + 1] - offs[idx[j]] : 0;
}

// Runs of 64 consecutive cycles of the new order per wavefront.  Their ids
// form one contiguous destination range, which the lanes copy word by
// word: lane l takes words l, l + 64, ..., and finds each word's cycle by
// walking forward through the run's destination offsets (kept in LDS), so
// every store is coalesced and every lane has work whatever the cycle
// lengths.  U words per lane are loaded before they are stored.
__global__ __launch_bounds__(CC_BLOCK) void k_gather_cycles(const unsigned *idx,
                                                            const long long *offs_old,
                                                            const int *verts_old,
                                                            const long long *offs_new,
                                                            int *verts_new, long long nc) {
  constexpr int U = 8;
  constexpr int NW = CC_BLOCK / CC_WAVE;
  __shared__ long long sSrc[NW][CC_WAVE];      // source offset of each cycle of the run
  __shared__ long long sDst[NW][CC_WAVE + 1];  // destination offsets, from the run's start
  const int lane = lane_id(), wave = threadIdx.x / CC_WAVE;
  const long long nw = (long long)gridDim.x * NW;
  for (long long j0 = ((long long)blockIdx.x * NW + wave) * CC_WAVE; j0 < nc;
       j0 += nw * CC_WAVE) {
    const int cnt = (int)min((long long)CC_WAVE, nc - j0);
    const long long j = j0 + lane;
    const long long d0 = (long long)uni_u64((unsigned long long)offs_new[j0]);
    if (lane < cnt) {
      sSrc[wave][lane] = offs_old[idx[j]];
      sDst[wave][lane] = offs_new[j] - d0;
    }
    if (lane == 0) sDst[wave][cnt] = offs_new[j0 + cnt] - d0;
    wave_lds_sync();
    const long long total = sDst[wave][cnt];
    int c = 0;  // the cycle of this lane's current word
    for (long long q0 = 0; q0 < total; q0 += (long long)U * CC_WAVE) {
      long long sa[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const long long q = q0 + (long long)u * CC_WAVE + lane;
        sa[u] = -1;
        if (q < total) {
          while (c + 1 < cnt && sDst[wave][c + 1] <= q) ++c;
          sa[u] = sSrc[wave][c] + (q - sDst[wave][c]);
        }
      }
      int val[U];
#pragma unroll
      for (int u = 0; u < U; ++u) val[u] = sa[u] >= 0 ? verts_old[sa[u]] : 0;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const long long q = q0 + (long long)u * CC_WAVE + lane;
        if (q < total) verts_new[d0 + q] = val[u];
      }
    }
    wave_lds_sync();  // the next run rewrites the offsets
  }
}

// first[r] = index of root r's first cycle in the sorted order (roots
// without cycles get the next root's), first[R] = nc.
__global__ void k_root_first(const unsigned *key, long long nc, long long R, long long *first) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x; j <= nc; j += stride) {
    const long long hi = j < nc ? min((long long)key[j], R) : R;
    const long long lo = j > 0 ? min((long long)key[j - 1], R) + 1 : 0;
    for (long long r = lo; r <= hi; ++r) first[r] = j;
  }
}


// Final histogram; in enumerate mode also closes the offsets array with the
// total vertex count.  One block.
__global__ void k_finalize(CcCtl *ctl, OutDev out, int n, int enumerate) {
  __shared__ unsigned long long sTot[CC_HSLOTS];
  finalize_body(ctl, out, n, enumerate != 0, sTot, CC_HSLOTS);
}

}  // namespace

// ------------------------------------------------------------------ launchers

hipError_t cc_launch_zero(void *p, size_t bytes, hipStream_t s) {
  const size_t words = bytes / 4;
  const int blocks = (int)min((size_t)1024, (words + 255) / 256 + 1);
  hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(256), 0, s, (unsigned int *)p, words);
  return hipGetLastError();
}

// Each launcher picks the instantiation for W = 1, 2, 4, 8 or 16 words per
// bitset (n <= 64, 128, 256, 512, 1024); batches take W <= 4.
#define CC_BY_W(W, F, ...)                                  \
  ((W) == 1 ? F<1>(__VA_ARGS__)                             \
   : (W) == 2 ? F<2>(__VA_ARGS__)                           \
   : (W) == 4 ? F<4>(__VA_ARGS__)                           \
   : (W) == 8 ? F<8>(__VA_ARGS__)                           \
   : (W) == 16 ? F<16>(__VA_ARGS__) : hipErrorInvalidValue)

namespace {
template <int W>
hipError_t launch_ingest(int n_graphs, const int *graph_vtx_off, int n_single, const int *row_ptr,
                         const int *col_idx, unsigned long long *adj, unsigned long long *adj_orig,
                         int *perm, int *label, unsigned int *status, long long *bound,
                         unsigned int *reply, hipStream_t s) {
  if (reply && n_graphs != 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_ingest<W>, dim3(n_graphs), dim3(128), 0, s, graph_vtx_off, n_single,
                     row_ptr, col_idx, adj, adj_orig, perm, label, status, bound, reply);
  return hipGetLastError();
}
template <int W>
hipError_t launch_triplets_batch(BatchDev bt, int n_graphs, hipStream_t s) {
  if (CC_BIG(W)) return hipErrorInvalidValue;  // batches hold graphs of at most 256 vertices
  hipLaunchKernelGGL(k_triplets_batch<CC_BIG(W) ? 4 : W>, dim3(n_graphs), dim3(CC_BLOCK), 0, s, bt);
  return hipGetLastError();
}
template <int W>
hipError_t step_occupancy(bool en, int *per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(
      per_cu, en ? (const void *)k_step<W, true> : (const void *)k_step<W, false>, CC_BLOCK, 0);
}
template <int W>
const void *head_fn(bool en) {
  return en ? (const void *)k_head<W, true> : (const void *)k_head<W, false>;
}
template <int W>
hipError_t head_raise(bool en, size_t lds_bytes) {
  return hipFuncSetAttribute(head_fn<W>(en), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)lds_bytes);
}
template <int W>
hipError_t launch_head(bool en, GraphDev g, CcCtl *ctl, const LevelBufs &b, OutDev out,
                       int forced_level, int cap, size_t lds_bytes, unsigned int *host_done,
                       int zero_cols, RootRange rr, hipStream_t s) {
  dim3 gr(1), bl(CC_HEAD_BLOCK(W));
  if (en) hipLaunchKernelGGL((k_head<W, true>), gr, bl, lds_bytes, s, g, ctl, b, out, forced_level, cap, host_done, zero_cols, rr);
  else hipLaunchKernelGGL((k_head<W, false>), gr, bl, lds_bytes, s, g, ctl, b, out, forced_level, cap, host_done, zero_cols, rr);
  return hipGetLastError();
}
template <int W>
hipError_t launch_root_total(GraphDev g, long long *out, hipStream_t s) {
  hipLaunchKernelGGL((k_root_total<W>), dim3(1), dim3(CC_BLOCK), 0, s, g, out);
  return hipGetLastError();
}
template <int W>
hipError_t launch_step(bool en, GraphDev g, CcCtl *ctl, const LevelBufs &b, OutDev out, int step,
                       int forced_level, int max_children, int allow_two, int blocks,
                       unsigned int *host_done, hipStream_t s) {
  dim3 gr(blocks), bl(CC_BLOCK);
  if (en) hipLaunchKernelGGL((k_step<W, true>), gr, bl, 0, s, g, ctl, b, out, step, forced_level, max_children, allow_two, host_done);
  else hipLaunchKernelGGL((k_step<W, false>), gr, bl, 0, s, g, ctl, b, out, step, forced_level, max_children, allow_two, host_done);
  return hipGetLastError();
}
template <int W>
hipError_t launch_dfs(bool en, GraphDev g, CcCtl *ctl, Frontier f0, Frontier f1, DfsWork wk,
                      OutDev out, unsigned long long *hist_out, int hist_stride, int cf,
                      int blocks, unsigned long long idle_timeout, hipStream_t s) {
  dim3 gr(blocks), bl(CC_BLOCK);
  const BatchDev nb{};
  if (en) hipLaunchKernelGGL((k_dfs<W, true, false>), gr, bl, 0, s, g, ctl, f0, f1, wk, out, hist_out, hist_stride, cf, idle_timeout, nb);
  else hipLaunchKernelGGL((k_dfs<W, false, false>), gr, bl, 0, s, g, ctl, f0, f1, wk, out, hist_out, hist_stride, cf, idle_timeout, nb);
  return hipGetLastError();
}
template <int W>
hipError_t dfs_occupancy(bool en, bool batch, int *per_cu) {
  const void *fn = batch ? (const void *)k_dfs<CC_BIG(W) ? 4 : W, false, true>
                         : en ? (const void *)k_dfs<W, true, false>
                              : (const void *)k_dfs<W, false, false>;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, fn, CC_BLOCK, 0);
}
template <int W>
hipError_t launch_dfs_batch(GraphDev g, CcCtl *ctl, DfsWork wk, BatchDev bt, int blocks,
                            unsigned long long idle_timeout, hipStream_t s) {
  if (CC_BIG(W)) return hipErrorInvalidValue;  // batches hold graphs of at most 256 vertices
  dim3 gr(blocks), bl(CC_BLOCK);
  const Frontier nf{};
  const OutDev no{};
  hipLaunchKernelGGL((k_dfs<CC_BIG(W) ? 4 : W, false, true>), gr, bl, 0, s, g, ctl, nf, nf, wk, no, nullptr, 0, 1, idle_timeout, bt);
  return hipGetLastError();
}
}  // namespace

hipError_t cc_launch_ingest(int W, int n_graphs, const int *graph_vtx_off, int n_single,
                            const int *row_ptr, const int *col_idx, unsigned long long *adj,
                            unsigned long long *adj_orig, int *perm, int *label,
                            unsigned int *status, long long *bound, unsigned int *reply,
                            hipStream_t s) {
  return CC_BY_W(W, launch_ingest, n_graphs, graph_vtx_off, n_single, row_ptr, col_idx, adj,
                 adj_orig, perm, label, status, bound, reply, s);
}

hipError_t cc_launch_triplets_batch(int W, BatchDev bt, int n_graphs, hipStream_t s) {
  if (n_graphs <= 0) return hipSuccess;
  return CC_BY_W(W, launch_triplets_batch, bt, n_graphs, s);
}


int cc_step_blocks_per_cu(int W, bool en) {
  // the same for every device of a process here (one architecture); asked
  // once per instantiation
  static std::atomic<int> cached[10];
  const int which = (W == 1 ? 0 : W == 2 ? 2 : W == 4 ? 4 : W == 8 ? 6 : 8) + (en ? 1 : 0);
  int v = cached[which].load();
  if (v <= 0) {
    int per_cu = 0;
    if (CC_BY_W(W, step_occupancy, en, &per_cu) != hipSuccess || per_cu <= 0) return 4;
    cached[which].store(per_cu);
    v = per_cu;
  }
  return v;
}

// Paths the head's LDS frontier buffers hold with `lds_bytes` of dynamic
// shared memory (two buffers).
int cc_head_capacity(int W, bool en, size_t lds_bytes) {
  const size_t per_path = (size_t)W * 8 * (en ? 2 : 1) + (W > 4 ? 4 : 2);
  long long cap = (long long)(lds_bytes / 2 / per_path) - 8;
  return cap > 0 ? (int)std::min<long long>(cap, 1 << 20) : 0;
}

hipError_t cc_launch_root_total(int W, GraphDev g, long long *out, hipStream_t s) {
  return CC_BY_W(W, launch_root_total, g, out, s);
}

hipError_t cc_launch_head(int W, bool en, GraphDev g, CcCtl *ctl, const LevelBufs &b,
                          OutDev out, int forced_level, size_t lds_bytes,
                          unsigned int *host_done, bool zero_ctl, RootRange roots,
                          hipStream_t s) {
  const int cap = cc_head_capacity(W, en, lds_bytes);
  const int zero_cols = zero_ctl ? std::min(std::max(g.n, 0) + 2, CC_HSLOTS) : 0;
  // The dynamic LDS limit is raised once per device and instantiation (the
  // call costs host time that would otherwise stall the stream).
  static std::atomic<size_t> raised[64][10];
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  const int which = (W == 1 ? 0 : W == 2 ? 2 : W == 4 ? 4 : W == 8 ? 6 : 8) + (en ? 1 : 0);
  if (dev >= 0 && dev < 64 && raised[dev][which].load() < lds_bytes) {
    e = CC_BY_W(W, head_raise, en, lds_bytes);
    if (e != hipSuccess) return e;
    raised[dev][which].store(lds_bytes);
  }
  return CC_BY_W(W, launch_head, en, g, ctl, b, out, forced_level, cap, lds_bytes, host_done,
                 zero_cols, roots, s);
}

// Static shared memory of the head kernel (so the caller can size the
// dynamic part).
size_t cc_head_static_lds(int W, bool en) {
  switch (W) {
    case 1: return en ? sizeof(HeadLds<1, true>) : sizeof(HeadLds<1, false>);
    case 2: return en ? sizeof(HeadLds<2, true>) : sizeof(HeadLds<2, false>);
    case 4: return en ? sizeof(HeadLds<4, true>) : sizeof(HeadLds<4, false>);
    case 8: return en ? sizeof(HeadLds<8, true>) : sizeof(HeadLds<8, false>);
    default: return en ? sizeof(HeadLds<16, true>) : sizeof(HeadLds<16, false>);
  }
}

hipError_t cc_launch_step(int W, bool en, GraphDev g, CcCtl *ctl, const LevelBufs &b,
                          OutDev out, int step, int forced_level, int max_children, bool two,
                          int blocks, unsigned int *host_done, hipStream_t s) {
  return CC_BY_W(W, launch_step, en, g, ctl, b, out, step, forced_level, max_children,
                 two ? 1 : 0, blocks, host_done, s);
}

hipError_t cc_launch_dfs(int W, bool en, GraphDev g, CcCtl *ctl, Frontier f0, Frontier f1,
                         DfsWork wk, OutDev out, unsigned long long *hist_out,
                         int hist_stride, bool count_front, int blocks,
                         unsigned long long idle_timeout, hipStream_t s) {
  return CC_BY_W(W, launch_dfs, en, g, ctl, f0, f1, wk, out, hist_out, hist_stride,
                 count_front ? 1 : 0, blocks, idle_timeout, s);
}

int cc_dfs_blocks_per_cu(int W, bool en, bool batch) {
  // asked once per instantiation (one architecture per process here)
  static std::atomic<int> cached[15];
  const int which = (W == 1 ? 0 : W == 2 ? 3 : W == 4 ? 6 : W == 8 ? 9 : 12) + (batch ? 2 : en ? 1 : 0);
  int v = cached[which].load();
  if (v <= 0) {
    int per_cu = 0;
    if (CC_BY_W(W, dfs_occupancy, en, batch, &per_cu) != hipSuccess ||
        per_cu <= 0)
      return 1;
    cached[which].store(per_cu);
    v = per_cu;
  }
  return v;
}

hipError_t cc_launch_dfs_batch(int W, GraphDev g, CcCtl *ctl, DfsWork wk, BatchDev bt, int blocks,
                               unsigned long long idle_timeout, hipStream_t s) {
  return CC_BY_W(W, launch_dfs_batch, g, ctl, wk, bt, blocks, idle_timeout, s);
}

namespace {
template <int W>
hipError_t launch_dfs_decode(GraphDev g, const CcCtl *ctl, OutDev out, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(k_dfs_decode<W>, dim3(blocks), dim3(CC_BLOCK), 0, s, g, ctl, out);
  return hipGetLastError();
}
}  // namespace

hipError_t cc_launch_dfs_decode(int W, GraphDev g, const CcCtl *ctl, OutDev out, int blocks,
                                hipStream_t s) {
  return CC_BY_W(W, launch_dfs_decode, g, ctl, out, std::max(1, blocks), s);
}

hipError_t cc_launch_dfs_prepare(CcCtl *ctl, DfsWork wk, int n, bool enum_bases, hipStream_t s) {
  const int blocks = std::max(1, std::min(1024, (wk.nwaves * 4 + 255) / 256));
  hipLaunchKernelGGL(k_dfs_prepare, dim3(blocks), dim3(256), 0, s, ctl, wk, n, enum_bases ? 1 : 0);
  return hipGetLastError();
}

hipError_t cc_launch_sort_cycles(const CcCtl *ctl, OutDev out, int n, int *tmp, unsigned *ia,
                                 unsigned *ib, hipStream_t s) {
  hipLaunchKernelGGL(k_sort_cycles, dim3(std::max(n + 1, 1)), dim3(kSortThreads), 0, s, ctl, out,
                     n, tmp, ia, ib);
  return hipGetLastError();
}

namespace {
// In-place exclusive scan of n int64 values; tmp holds cc_scan_tmp(n) words.
hipError_t scan_exclusive(long long *x, long long n, long long *tmp, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const long long nb = (n + kScanTile - 1) / kScanTile;
  if (nb == 1) {
    hipLaunchKernelGGL(k_scan_tile, dim3(1), dim3(kScanThreads), 0, s, x, n, nullptr);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_scan_tile, dim3((unsigned)nb), dim3(kScanThreads), 0, s, x, n, tmp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = scan_exclusive(tmp, nb, tmp + nb, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(kScanThreads), 0, s, x, n, tmp);
  return hipGetLastError();
}
long long scan_tmp_words(long long n) {
  long long w = 0;
  while (n > kScanTile) {
    n = (n + kScanTile - 1) / kScanTile;
    w += n;
  }
  return w + 1;
}
template <int W>
hipError_t launch_group_roots(GraphDev g, const int *label, const int *verts_old,
                              const long long *offs_old, long long nc, long long R,
                              int *verts_new, long long *offs_new, long long *first, char *work,
                              hipStream_t s) {
  const long long nb = std::max(1ll, (nc + kRsTile - 1) / kRsTile);
  auto take = [&](size_t bytes) {
    char *p = work;
    work += (bytes + 255) / 256 * 256;
    return p;
  };
  long long *root_base = (long long *)take((size_t)CC_MAXN * 8);
  unsigned *ka = (unsigned *)take((size_t)std::max(nc, 1ll) * 4);
  unsigned *ia = (unsigned *)take((size_t)std::max(nc, 1ll) * 4);
  unsigned *kb = (unsigned *)take((size_t)std::max(nc, 1ll) * 4);
  unsigned *ib = (unsigned *)take((size_t)std::max(nc, 1ll) * 4);
  long long *table = (long long *)take((size_t)(256 * nb) * 8);
  long long *tmp = (long long *)take((size_t)scan_tmp_words(std::max(256 * nb, nc + 1)) * 8);
  hipLaunchKernelGGL(k_root_base<W>, dim3(1), dim3(64), 0, s, g, label, root_base);
  const unsigned kb_blocks = (unsigned)std::min(std::max(1ll, (nc + CC_BLOCK - 1) / CC_BLOCK), 8192ll);
  hipLaunchKernelGGL(k_cycle_root_keys<W>, dim3(kb_blocks), dim3(CC_BLOCK), 0, s, g, label,
                     root_base, verts_old, offs_old, nc, R, ka, ia);
  hipError_t e = hipGetLastError();
  // enough 8-bit digits for keys up to R (malformed cycles carry R)
  int passes = 1;
  while (passes < 4 && (R >> (8 * passes)) != 0) ++passes;
  for (int p = 0; p < passes && e == hipSuccess && nc > 0; ++p) {
    hipLaunchKernelGGL(k_rs_count, dim3((unsigned)nb), dim3(kRsThreads), 0, s, ka, nc, 8 * p,
                       table, (int)nb);
    e = hipGetLastError();
    if (e == hipSuccess) e = scan_exclusive(table, 256 * nb, tmp, s);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(k_rs_scatter, dim3((unsigned)nb), dim3(kRsThreads), 0, s, ka, ia, kb, ib,
                         nc, 8 * p, table, (int)nb);
      e = hipGetLastError();
    }
    std::swap(ka, kb);
    std::swap(ia, ib);
  }
  if (e != hipSuccess) return e;
  const unsigned lb = (unsigned)std::min(std::max(1ll, (nc + 1 + 255) / 256), 16384ll);
  hipLaunchKernelGGL(k_sorted_lengths, dim3(lb), dim3(256), 0, s, ia, offs_old, nc, offs_new);
  e = hipGetLastError();
  if (e == hipSuccess) e = scan_exclusive(offs_new, nc + 1, tmp, s);
  if (e != hipSuccess) return e;
  const unsigned gb = (unsigned)std::min(std::max(1ll, (nc + CC_BLOCK - 1) / CC_BLOCK), 8192ll);
  hipLaunchKernelGGL(k_gather_cycles, dim3(gb), dim3(CC_BLOCK), 0, s, ia, offs_old, verts_old,
                     offs_new, verts_new, nc);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const unsigned fb = (unsigned)std::min(std::max(1ll, (nc + 1 + 255) / 256), 16384ll);
  hipLaunchKernelGGL(k_root_first, dim3(fb), dim3(256), 0, s, ka, nc, R, first);
  return hipGetLastError();
}
}  // namespace

size_t cc_group_roots_workspace(long long nc) {
  const long long nb = std::max(1ll, (nc + kRsTile - 1) / kRsTile);
  const size_t c = (size_t)std::max(nc, 1ll);
  auto a = [](size_t b) { return (b + 255) / 256 * 256; };
  return a((size_t)CC_MAXN * 8) + 4 * a(c * 4) + a((size_t)(256 * nb) * 8) +
         a((size_t)scan_tmp_words(std::max(256 * nb, nc + 1)) * 8);
}

hipError_t cc_launch_group_roots(int W, GraphDev g, const int *label, const int *verts_old,
                                 const long long *offs_old, long long nc, long long R,
                                 int *verts_new, long long *offs_new, long long *first, void *work,
                                 hipStream_t s) {
  return CC_BY_W(W, launch_group_roots, g, label, verts_old, offs_old, nc, R, verts_new, offs_new,
                 first, (char *)work, s);
}

hipError_t cc_launch_finalize(CcCtl *ctl, OutDev out, int n, bool en, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, s, ctl, out, n, en ? 1 : 0);
  return hipGetLastError();
}
