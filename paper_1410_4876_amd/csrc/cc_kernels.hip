// HIP kernels for chordless-cycle enumeration on gfx950 (MI355X).
//
// Vertices are renumbered by their degree label (Section 2), so "label
// greater than the label of v2" is an integer comparison and every vertex
// set is a W-word bitset (W = ceil(n / 64), n <= 128).  An open chordless
// path p = <v1, ..., vt> is carried as (X, S, v1, vt) where
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
template <int W>
__device__ __forceinline__ bool btest(Bits<W> a, int v) {
  unsigned long long word = a.w[0];
  if (W == 2 && v >= 64) word = a.w[W - 1];
  return (word >> (v & 63)) & 1ull;
}
template <int W>
__device__ __forceinline__ Bits<W> bsingle(int v) {
  Bits<W> a = bzero<W>();
  if (W == 1 || v < 64) a.w[0] = 1ull << (v & 63);
  else a.w[W - 1] = 1ull << (v & 63);
  return a;
}
// Lowest set bit index (a must be non-empty); clears it.
template <int W>
__device__ __forceinline__ int bpop_lowest(Bits<W> &a) {
  if (W == 1 || a.w[0]) {
    int v = __ffsll((long long)a.w[0]) - 1;
    a.w[0] &= a.w[0] - 1ull;
    return v;
  }
  int v = __ffsll((long long)a.w[W - 1]) - 1;
  a.w[W - 1] &= a.w[W - 1] - 1ull;
  return 64 + v;
}
// {w : w <= u}
template <int W>
__device__ __forceinline__ Bits<W> low_through(int u) {
  Bits<W> a;
  if (W == 1) {
    a.w[0] = (u >= 63) ? ~0ull : ((2ull << u) - 1ull);
  } else {
    if (u >= 64) {
      a.w[0] = ~0ull;
      a.w[W - 1] = (u >= 127) ? ~0ull : ((2ull << (u - 64)) - 1ull);
    } else {
      a.w[0] = (u >= 63) ? ~0ull : ((2ull << u) - 1ull);
      a.w[W - 1] = 0ull;
    }
  }
  return a;
}

// ------------------------------------------------------- wave primitives
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ unsigned long long wave_ballot(bool p) { return __ballot(p); }

// Number of set bits of `mask` at lanes below this one.
__device__ __forceinline__ unsigned int lanes_below(unsigned long long mask) {
  return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

__device__ __forceinline__ unsigned int wave_sum_u32(unsigned int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, CC_WAVE);
  return v;
}
__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, CC_WAVE);
  return v;
}
__device__ __forceinline__ unsigned int wave_min_u32(unsigned int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, CC_WAVE));
  return v;
}
__device__ __forceinline__ unsigned long long bcast_u64(unsigned long long v) {
  return __shfl(v, 0, CC_WAVE);
}
__device__ __forceinline__ long long bcast_i64(long long v) { return __shfl(v, 0, CC_WAVE); }

template <typename T>
__device__ __forceinline__ T ld_acquire(T *p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_release(T *p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// -------------------------------------------------------------- decoding
// Writes the k vertices of the chordless cycle C (label-space bitset) as
// original ids, starting at the smallest original id and continuing towards
// the smaller of its two cycle neighbours.  In an induced cycle every vertex
// has exactly two neighbours inside C, so the walk is unique.
template <int W>
__device__ void write_cycle(const unsigned long long *sN, const int *sPerm, Bits<W> C, int k,
                            int *dst) {
  Bits<W> it = C;
  int start = -1, best = 0x7fffffff;
  while (bany(it)) {
    int v = bpop_lowest(it);
    int o = sPerm[v];
    if (o < best) {
      best = o;
      start = v;
    }
  }
  Bits<W> nb = band(row<W>(sN, start), C);
  const int a = bany(nb) ? bpop_lowest(nb) : start;
  const int b = bany(nb) ? bpop_lowest(nb) : a;
  int cur = (sPerm[a] < sPerm[b]) ? a : b;
  int prev = start;
  dst[0] = best;
  dst[1] = sPerm[cur];
  for (int j = 2; j < k; ++j) {
    Bits<W> nx = band(row<W>(sN, cur), bandnot(C, bsingle<W>(prev)));
    const int nxt = bany(nx) ? bpop_lowest(nx) : start;  // C is always a cycle here
    dst[j] = sPerm[nxt];
    prev = cur;
    cur = nxt;
  }
}

// ----------------------------------------------------------------- zero
__global__ void k_zero(unsigned int *p, size_t words) {
  size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < words; i += stride) p[i] = 0u;
}

// --------------------------------------------------------------- ingest
// One block per graph.  Validates the CSR (simple, symmetric), builds the
// adjacency bitsets, computes the degree labelling (Section 2: repeatedly
// take the remaining vertex of minimum remaining degree, smallest id on
// ties; it gets the next label) with one wavefront holding two vertices per
// lane, and writes the bitsets renumbered by label.
template <int W>
__global__ __launch_bounds__(128) void k_ingest(const int *__restrict__ graph_vtx_off,
                                                int n_single, const int *__restrict__ rp,
                                                const int *__restrict__ ci,
                                                unsigned long long *__restrict__ adj_out,
                                                int *__restrict__ perm_out,
                                                int *__restrict__ label_out,
                                                unsigned int *__restrict__ status) {
  __shared__ unsigned long long sA[CC_MAXN * W];
  __shared__ int sLab[CC_MAXN];
  __shared__ unsigned int sErr;
  __shared__ unsigned int sDeg;
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
  }
  for (int i = tid; i < CC_MAXN * W; i += blockDim.x) sA[i] = 0ull;
  __syncthreads();
  if (n < 0 || n > 64 * W) {
    if (tid == 0) status[g] = CC_DEV_NOT_SIMPLE;
    return;
  }
  const long long e0 = rp[v0];
  const long long eN = rp[v0 + n];
  const bool bad_head = (v0 == 0 && e0 != 0) || eN < e0 || (eN - e0) > (long long)n * (n - 1);
  if (bad_head) {
    if (tid == 0) status[g] = CC_DEV_NOT_SIMPLE;
    return;
  }
  for (int v = tid; v < n; v += blockDim.x) {
    const long long a = rp[v0 + v], b = rp[v0 + v + 1];
    if (b < a || a < e0 || b > eN) {
      atomicOr(&sErr, CC_DEV_NOT_SIMPLE);
      continue;
    }
    unsigned long long r0 = 0ull, r1 = 0ull;
    bool bad = false;
    for (long long e = a; e < b && !bad; ++e) {
      const int w = ci[e] - v0;
      if (w < 0 || w >= n || w == v) {
        bad = true;
        break;
      }
      const unsigned long long bit = 1ull << (w & 63);
      if (w < 64) {
        bad = (r0 & bit) != 0ull;
        r0 |= bit;
      } else {
        bad = (r1 & bit) != 0ull;
        r1 |= bit;
      }
    }
    if (bad) atomicOr(&sErr, CC_DEV_NOT_SIMPLE);
    sA[v * W] = r0;
    if (W == 2) sA[v * W + W - 1] = r1;
    atomicMax(&sDeg, (unsigned)(b - a));
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
    if (tid == 0) status[g] = sErr;
    return;
  }
  if (tid < CC_WAVE) {
    const int va = tid, vb = tid + CC_WAVE;
    int dega = va < n ? bpop(row<W>(sA, va)) : 0;
    int degb = vb < n ? bpop(row<W>(sA, vb)) : 0;
    bool alivea = va < n, aliveb = vb < n;
    for (int i = 0; i < n; ++i) {
      unsigned ka = alivea ? (((unsigned)dega << 8) | (unsigned)va) : 0xffffffffu;
      unsigned kb = aliveb ? (((unsigned)degb << 8) | (unsigned)vb) : 0xffffffffu;
      const unsigned key = wave_min_u32(min(ka, kb));
      const int u = (int)(key & 0xffu);
      if (va == u) {
        alivea = false;
        sLab[u] = i;
      }
      if (vb == u) {
        aliveb = false;
        sLab[u] = i;
      }
      if (alivea && btest(row<W>(sA, va), u)) --dega;
      if (aliveb && btest(row<W>(sA, vb), u)) --degb;
    }
  }
  __syncthreads();
  for (int v = tid; v < n; v += blockDim.x) {
    const int l = sLab[v];
    perm_out[v0 + l] = v;
    label_out[v0 + v] = l;
    Bits<W> r = row<W>(sA, v);
    Bits<W> out = bzero<W>();
    while (bany(r)) out = bor(out, bsingle<W>(sLab[bpop_lowest(r)]));
#pragma unroll
    for (int k = 0; k < W; ++k) adj_out[(size_t)(v0 + l) * W + k] = out.w[k];
  }
  if (tid == 0) status[g] = 0x100u | (sDeg << 16);  // bit 8: ok; bits 16..: max degree
}

// ------------------------------------------------------------- stage one
// Initial triplets and triangles (Algorithm 1's set T(G) and the triangles
// of C; Algorithm 2 computes the same sets).  One block; each thread takes
// (u, x) pairs with x a higher-labelled neighbour of u and scans the
// neighbours y of u above x.
template <int W, bool ENUM>
__global__ __launch_bounds__(CC_BLOCK) void k_triplets(GraphDev g, CcCtl *ctl, Frontier f,
                                                       OutDev out) {
  __shared__ unsigned long long sN[CC_MAXN * W];
  __shared__ int sPerm[CC_MAXN];
  __shared__ unsigned long long sRed[CC_BLOCK / CC_WAVE];
  const int n = g.n;
  const int tid = threadIdx.x;
  for (int i = tid; i < n * W; i += CC_BLOCK) sN[i] = g.adj[i];
  for (int i = tid; i < n; i += CC_BLOCK) sPerm[i] = g.perm[i];
  __syncthreads();
  unsigned long long tri = 0;
  for (int idx = tid; idx < n * n; idx += CC_BLOCK) {
    const int u = idx / n, x = idx - u * n;
    const Bits<W> nu = row<W>(sN, u);
    if (x <= u || !btest(nu, x)) continue;
    const Bits<W> nx = row<W>(sN, x);
    Bits<W> ys = bandnot(nu, low_through<W>(x));
    while (bany(ys)) {
      const int y = bpop_lowest(ys);
      if (btest(nx, y)) {
        if (ENUM) {
          const unsigned long long slot = atomicAdd(&ctl->hist[3], 1ull);
          const long long pos = (long long)slot * 3;
          if ((long long)slot < out.cyc_cap && pos + 3 <= out.verts_cap) {
            Bits<W> C = bor(bor(bsingle<W>(x), bsingle<W>(u)), bsingle<W>(y));
            write_cycle<W>(sN, sPerm, C, 3, out.verts + pos);
            out.offs[slot] = pos;
          }
        } else {
          ++tri;
        }
      } else {
        const unsigned long long slot = atomicAdd(&ctl->count[3], 1ull);
        if (slot < f.cap) {
          const Bits<W> X = bor(nu, low_through<W>(u));
#pragma unroll
          for (int k = 0; k < W; ++k) f.X[k * f.cap + slot] = X.w[k];
          if (ENUM) {
            const Bits<W> S = bor(bor(bsingle<W>(x), bsingle<W>(u)), bsingle<W>(y));
#pragma unroll
            for (int k = 0; k < W; ++k) f.S[k * f.cap + slot] = S.w[k];
          }
          f.vv[slot] = (unsigned short)(x | (y << 8));
        }
      }
    }
  }
  if (!ENUM) {
    tri = wave_sum_u64(tri);
    if (lane_id() == 0) sRed[tid / CC_WAVE] = tri;
    __syncthreads();
    if (tid == 0) {
      unsigned long long s = 0;
      for (int i = 0; i < CC_BLOCK / CC_WAVE; ++i) s += sRed[i];
      if (s) atomicAdd(&ctl->hist[3], s);
    }
  }
}

// ------------------------------------------------------ breadth-first level
// One level of Algorithm 3 over the frontier of paths with t vertices:
// every path is expanded by one lane; closures are counted into hist[t+1]
// (and written, enumerate mode); extensions are compacted into the next
// frontier with one atomic per wavefront plus ballot/mbcnt ranks.  The
// frontier size lives in device memory (count[t]), so the host launches the
// level loop without reading anything back (Algorithm 4's fixed relaunches).
template <int W, bool ENUM>
__global__ __launch_bounds__(CC_BLOCK) void k_level(GraphDev g, CcCtl *ctl, Frontier fin,
                                                    Frontier fout, OutDev out, int t,
                                                    int forced_level) {
  __shared__ unsigned long long sN[CC_MAXN * W];
  __shared__ int sPerm[ENUM ? CC_MAXN : 1];
  __shared__ unsigned long long sRed[CC_BLOCK / CC_WAVE];
  __shared__ long long sBase[2];
  if (ld_acquire(&ctl->mode) != 0) return;
  const unsigned long long cnt = ctl->count[t];
  if (cnt > fin.cap) {
    // The previous level produced more paths than fit: hand its (intact)
    // input frontier to the depth-first kernel; that level's closures and
    // path count are already recorded.
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      ctl->skip_first = 1;
      ctl->switch_level = t - 1;
      ctl->bfs_max_len = t;
      __threadfence();
      st_release(&ctl->mode, 1);
    }
    return;
  }
  if (t == forced_level) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      ctl->skip_first = 0;
      ctl->switch_level = t;
      ctl->bfs_max_len = t;
      __threadfence();
      st_release(&ctl->mode, 1);
    }
    return;
  }
  if (cnt == 0) return;
  const int n = g.n;
  const int tid = threadIdx.x;
  for (int i = tid; i < n * W; i += CC_BLOCK) sN[i] = g.adj[i];
  if (ENUM) {
    for (int i = tid; i < n; i += CC_BLOCK) sPerm[i] = g.perm[i];
    if (tid == 0) {
      long long cb = 0, vb = 0;
      for (int j = 3; j <= t; ++j) {
        cb += (long long)ctl->hist[j];
        vb += (long long)ctl->hist[j] * j;
      }
      sBase[0] = cb;
      sBase[1] = vb;
    }
  }
  __syncthreads();
  if (blockIdx.x == 0 && tid == 0) {
    ctl->front[t] = cnt;
    atomicMax(&ctl->peak, cnt);
  }
  const int lane = lane_id();
  const unsigned long long nwaves = (unsigned long long)gridDim.x * (CC_BLOCK / CC_WAVE);
  const unsigned long long wv = (unsigned long long)blockIdx.x * (CC_BLOCK / CC_WAVE) + tid / CC_WAVE;
  const int k = t + 1;
  unsigned long long acc = 0;
  for (unsigned long long b0 = wv * CC_WAVE; b0 < cnt; b0 += nwaves * CC_WAVE) {
    const unsigned long long i = b0 + lane;
    const bool valid = i < cnt;
    Bits<W> X = bzero<W>(), S = bzero<W>();
    int v1 = 0, vt = 0;
    if (valid) {
#pragma unroll
      for (int w = 0; w < W; ++w) X.w[w] = fin.X[w * fin.cap + i];
      if (ENUM) {
#pragma unroll
        for (int w = 0; w < W; ++w) S.w[w] = fin.S[w * fin.cap + i];
      }
      const unsigned vv = fin.vv[i];
      v1 = vv & 0xffu;
      vt = vv >> 8;
    }
    const Bits<W> nvt = row<W>(sN, vt);
    const Bits<W> nv1 = row<W>(sN, v1);
    const Bits<W> cand = bandnot(nvt, X);
    Bits<W> clos = band(cand, nv1);
    Bits<W> ext = bandnot(cand, nv1);
    if (!valid) {
      clos = bzero<W>();
      ext = bzero<W>();
    }
    if (ENUM) {
      const unsigned tot = wave_sum_u32((unsigned)bpop(clos));
      if (tot) {
        unsigned long long slot0 = 0;
        if (lane == 0) slot0 = atomicAdd(&ctl->hist[k], (unsigned long long)tot);
        slot0 = bcast_u64(slot0);
        unsigned long long off = 0;
        while (true) {
          const bool has = bany(clos);
          const unsigned long long mask = wave_ballot(has);
          if (!mask) break;
          if (has) {
            const int v = bpop_lowest(clos);
            const unsigned long long slot = slot0 + off + lanes_below(mask);
            const long long cyc = sBase[0] + (long long)slot;
            const long long pos = sBase[1] + (long long)slot * k;
            if (cyc < out.cyc_cap && pos + k <= out.verts_cap) {
              write_cycle<W>(sN, sPerm, bor(S, bsingle<W>(v)), k, out.verts + pos);
              out.offs[cyc] = pos;
            }
          }
          off += __popcll(mask);
        }
      }
    } else {
      acc += (unsigned long long)bpop(clos);
    }
    const unsigned tot = wave_sum_u32((unsigned)bpop(ext));
    if (tot) {
      unsigned long long slot0 = 0;
      if (lane == 0) slot0 = atomicAdd(&ctl->count[k], (unsigned long long)tot);
      slot0 = bcast_u64(slot0);
      const Bits<W> Xn = bor(X, nvt);
      unsigned long long off = 0;
      while (true) {
        const bool has = bany(ext);
        const unsigned long long mask = wave_ballot(has);
        if (!mask) break;
        if (has) {
          const int v = bpop_lowest(ext);
          const unsigned long long slot = slot0 + off + lanes_below(mask);
          if (slot < fout.cap) {
#pragma unroll
            for (int w = 0; w < W; ++w) fout.X[w * fout.cap + slot] = Xn.w[w];
            if (ENUM) {
              const Bits<W> Sn = bor(S, bsingle<W>(v));
#pragma unroll
              for (int w = 0; w < W; ++w) fout.S[w * fout.cap + slot] = Sn.w[w];
            }
            fout.vv[slot] = (unsigned short)(v1 | (v << 8));
          }
        }
        off += __popcll(mask);
      }
    }
  }
  if (!ENUM) {
    acc = wave_sum_u64(acc);
    if (lane == 0) sRed[tid / CC_WAVE] = acc;
    __syncthreads();
    if (tid == 0) {
      unsigned long long s = 0;
      for (int i = 0; i < CC_BLOCK / CC_WAVE; ++i) s += sRed[i];
      if (s) atomicAdd(&ctl->hist[k], s);
    }
  }
}

// ---------------------------------------------------------- depth-first
// Donation queue: a bounded multi-producer multi-consumer ring of chunks
// (each up to CC_CHUNK paths) with one sequence number per cell.  Only lane
// 0 of a wavefront touches the cursors; the whole wavefront moves the data.
__device__ long long q_reserve_push(CcCtl *ctl, const DfsWork &wk) {
  unsigned long long pos = ld_acquire(&ctl->q_tail);
  for (int attempt = 0; attempt < 32; ++attempt) {
    const unsigned long long cell = pos & (wk.qcap - 1);
    const unsigned long long seq = ld_acquire(&wk.qseq[cell]);
    const long long diff = (long long)(seq - pos);
    if (diff == 0) {
      if (atomicCAS(&ctl->q_tail, pos, pos + 1) == pos) return (long long)pos;
      pos = ld_acquire(&ctl->q_tail);
    } else if (diff < 0) {
      return -1;  // full
    } else {
      pos = ld_acquire(&ctl->q_tail);
    }
  }
  return -1;
}

__device__ long long q_reserve_pop(CcCtl *ctl, const DfsWork &wk) {
  unsigned long long pos = ld_acquire(&ctl->q_head);
  for (int attempt = 0; attempt < 32; ++attempt) {
    const unsigned long long cell = pos & (wk.qcap - 1);
    const unsigned long long seq = ld_acquire(&wk.qseq[cell]);
    const long long diff = (long long)(seq - (pos + 1));
    if (diff == 0) {
      if (atomicCAS(&ctl->q_head, pos, pos + 1) == pos) return (long long)pos;
      pos = ld_acquire(&ctl->q_head);
    } else if (diff < 0) {
      return -1;  // empty
    } else {
      pos = ld_acquire(&ctl->q_head);
    }
  }
  return -1;
}

__device__ __forceinline__ bool work_visible(CcCtl *ctl, unsigned long long nroots) {
  if (ld_acquire(&ctl->root_cursor) < nroots) return true;
  const unsigned long long h = ld_acquire(&ctl->q_head);
  const unsigned long long tl = ld_acquire(&ctl->q_tail);
  return tl > h;
}

// Depth-first continuation (north of the memory budget).  Each wavefront
// owns a LIFO stack of open paths in device memory; a step pops up to 64
// paths (one per lane), expands them exactly like a breadth-first level and
// pushes the extensions back, so memory grows with depth, not with the
// frontier.  Work enters from the handed-over frontier (claimed in chunks of
// 64 with an atomic cursor) and from chunks that busy wavefronts donate from
// the bottom of their stacks when others are idle.  Termination: a
// wavefront leaves only after it saw no busy wavefront and then no visible
// work; a wavefront holding paths is always counted busy.
template <int W, bool ENUM>
__global__ __launch_bounds__(CC_BLOCK) void k_dfs(GraphDev g, CcCtl *ctl, Frontier f0,
                                                  Frontier f1, DfsWork wk0, DfsWork wk1,
                                                  OutDev out, unsigned long long *hist_out,
                                                  int count_front,
                                                  unsigned long long idle_timeout) {
  __shared__ unsigned long long sN[CC_MAXN * W];
  __shared__ int sPerm[ENUM ? CC_MAXN : 1];
  __shared__ unsigned long long sHist[CC_HSLOTS];
  __shared__ unsigned long long sFront[CC_HSLOTS];
  __shared__ long long sCb[ENUM ? CC_HSLOTS : 1];
  __shared__ long long sVb[ENUM ? CC_HSLOTS : 1];
  if (ld_acquire(&ctl->mode) == 0) return;
  const int L = ctl->switch_level;
  const bool skip = ctl->skip_first != 0;
  const Frontier roots = (L & 1) ? f1 : f0;
  const DfsWork wk = (L & 1) ? wk0 : wk1;  // the buffer not holding the roots
  const unsigned long long nroots = min(ctl->count[L], roots.cap);
  const int n = g.n;
  const int tid = threadIdx.x;
  for (int i = tid; i < n * W; i += CC_BLOCK) sN[i] = g.adj[i];
  for (int i = tid; i < CC_HSLOTS; i += CC_BLOCK) {
    sHist[i] = 0ull;
    sFront[i] = 0ull;
  }
  if (ENUM) {
    for (int i = tid; i < n; i += CC_BLOCK) sPerm[i] = g.perm[i];
    for (int i = tid; i < CC_HSLOTS; i += CC_BLOCK) {
      sCb[i] = (long long)ctl->len_cbase[i];
      sVb[i] = (long long)ctl->len_vbase[i];
    }
  }
  __syncthreads();

  const int lane = lane_id();
  const unsigned long long wid = (unsigned long long)blockIdx.x * (CC_BLOCK / CC_WAVE) + tid / CC_WAVE;
  const unsigned long long cap = wk.cap_w;
  unsigned long long *stX = wk.stackX + wid * W * cap;
  unsigned long long *stS = ENUM ? wk.stackS + wid * W * cap : nullptr;
  unsigned int *stM = wk.stackM + wid * cap;
  const unsigned long long maxc = (unsigned long long)max(wk.max_children, 1);

  unsigned long long bot = 0, top = 0;
  unsigned long long steps = 0, batches = 0, donated = 0;
  if (lane == 0) atomicAdd(&ctl->busy, 1);

  while (true) {
    Bits<W> X = bzero<W>(), S = bzero<W>();
    unsigned int m = 0;
    bool valid = false;
    if (top > bot) {
      // Pop up to 64 paths from the top, keeping room for their extensions.
      unsigned long long kk = min(top - bot, (unsigned long long)CC_CHUNK);
      while (kk > 1 && (top - kk) + kk * maxc > cap) kk >>= 1;
      const unsigned long long start = top - kk;
      valid = (unsigned long long)lane < kk;
      if (valid) {
        const unsigned long long i = start + lane;
#pragma unroll
        for (int w = 0; w < W; ++w) X.w[w] = stX[w * cap + i];
        if (ENUM) {
#pragma unroll
          for (int w = 0; w < W; ++w) S.w[w] = stS[w * cap + i];
        }
        m = stM[i];
      }
      top = start;
      if (top == bot) top = bot = 0;
    } else {
      bool got = false;
      // 1. the handed-over frontier
      if (ld_acquire(&ctl->root_cursor) < nroots) {
        unsigned long long c = 0;
        if (lane == 0) c = atomicAdd(&ctl->root_cursor, (unsigned long long)CC_CHUNK);
        c = bcast_u64(c);
        if (c < nroots) {
          const unsigned long long kk = min(nroots - c, (unsigned long long)CC_CHUNK);
          valid = (unsigned long long)lane < kk;
          if (valid) {
            const unsigned long long i = c + lane;
#pragma unroll
            for (int w = 0; w < W; ++w) X.w[w] = roots.X[w * roots.cap + i];
            if (ENUM) {
#pragma unroll
              for (int w = 0; w < W; ++w) S.w[w] = roots.S[w * roots.cap + i];
            }
            const unsigned vv = roots.vv[i];
            m = (vv & 0xffu) | ((vv >> 8) << 8) | ((unsigned)L << 16) | (1u << 24);
          }
          got = true;
        }
      }
      // 2. a donated chunk
      if (!got) {
        long long pos = -1;
        if (lane == 0) pos = q_reserve_pop(ctl, wk);
        pos = bcast_i64(pos);
        if (pos >= 0) {
          const unsigned long long cell = (unsigned long long)pos & (wk.qcap - 1);
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
          const unsigned kk = wk.qN[cell];
          valid = (unsigned)lane < kk;
          if (valid) {
            const unsigned long long base = cell * CC_CHUNK + lane;
#pragma unroll
            for (int w = 0; w < W; ++w) X.w[w] = wk.qX[(cell * W + w) * CC_CHUNK + lane];
            if (ENUM) {
#pragma unroll
              for (int w = 0; w < W; ++w) S.w[w] = wk.qS[(cell * W + w) * CC_CHUNK + lane];
            }
            m = wk.qM[base];
          }
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
          if (lane == 0) st_release(&wk.qseq[cell], (unsigned long long)pos + wk.qcap);
          got = true;
        }
      }
      // 3. nothing anywhere: wait as idle, or leave
      if (!got) {
        if (lane == 0) {
          atomicSub(&ctl->busy, 1);
          atomicAdd(&ctl->idle, 1);
        }
        bool leave = false;
        const unsigned long long t0 = wall_clock64();
        while (true) {
          __builtin_amdgcn_s_sleep(8);
          int flag = 0;  // 1: work seen, 2: leave
          if (lane == 0) {
            if (work_visible(ctl, nroots)) {
              flag = 1;
            } else if (ld_acquire(&ctl->busy) == 0) {
              flag = work_visible(ctl, nroots) ? 1 : 2;
            } else if (wall_clock64() - t0 > idle_timeout) {
              flag = 3;
            }
          }
          flag = __shfl(flag, 0, CC_WAVE);
          if (flag == 1) {
            if (lane == 0) {
              atomicAdd(&ctl->busy, 1);
              atomicSub(&ctl->idle, 1);
            }
            break;
          }
          if (flag >= 2) {
            if (lane == 0) {
              atomicSub(&ctl->idle, 1);
              if (flag == 3) atomicOr(&ctl->status, CC_DEV_IDLE_TIMEOUT);
            }
            leave = true;
            break;
          }
        }
        if (leave) break;
        continue;
      }
    }

    // ---- expand the batch (one path per lane)
    ++batches;
    const int v1 = m & 0xffu;
    const int vt = (m >> 8) & 0xffu;
    const int t = (m >> 16) & 0xffu;
    const bool first = valid && (m >> 24) && skip;
    const Bits<W> nvt = row<W>(sN, vt);
    const Bits<W> nv1 = row<W>(sN, v1);
    const Bits<W> cand = bandnot(nvt, X);
    Bits<W> clos = band(cand, nv1);
    Bits<W> ext = bandnot(cand, nv1);
    if (!valid) {
      clos = bzero<W>();
      ext = bzero<W>();
    }
    if (valid && !first) {
      if (count_front) atomicAdd(&sFront[t], 1ull);
      const int c = bpop(clos);
      if (c) {
        if (hist_out) atomicAdd(&sHist[t + 1], (unsigned long long)c);
        if (ENUM) {
          const int k = t + 1;
          const unsigned long long slot0 = atomicAdd(&ctl->len_cursor[k], (unsigned long long)c);
          Bits<W> cl = clos;
          for (int j = 0; j < c; ++j) {
            const int v = bpop_lowest(cl);
            const long long cyc = sCb[k] + (long long)(slot0 + j);
            const long long pos = sVb[k] + (long long)(slot0 + j) * k;
            if (cyc < out.cyc_cap && pos + k <= out.verts_cap) {
              write_cycle<W>(sN, sPerm, bor(S, bsingle<W>(v)), k, out.verts + pos);
              out.offs[cyc] = pos;
            }
          }
        }
      }
    }
    // A path never has more than n vertices (each extension adds a vertex
    // outside S, and S is inside X); anything longer would mean corrupted
    // state, so it is dropped and reported instead of looping.
    if (t >= n && bany(ext)) {
      atomicOr(&ctl->status, CC_DEV_STACK_FULL);
      ext = bzero<W>();
    }
    const unsigned tot = wave_sum_u32((unsigned)bpop(ext));
    if (tot) {
      if (top + tot > cap && bot > 0) {
        // Slide the live part of the stack down to index 0 (chunks of 64;
        // bot is a multiple of 64, so a chunk never overlaps its source).
        const unsigned long long live = top - bot;
        for (unsigned long long c0 = 0; c0 < live; c0 += CC_CHUNK) {
          const unsigned long long i = c0 + lane;
          if (i < live) {
#pragma unroll
            for (int w = 0; w < W; ++w) stX[w * cap + i] = stX[w * cap + bot + i];
            if (ENUM) {
#pragma unroll
              for (int w = 0; w < W; ++w) stS[w * cap + i] = stS[w * cap + bot + i];
            }
            stM[i] = stM[bot + i];
          }
        }
        top = live;
        bot = 0;
      }
      if (top + tot > cap) {
        if (lane == 0) atomicOr(&ctl->status, CC_DEV_STACK_FULL);
      } else {
        const Bits<W> Xn = bor(X, nvt);
        const unsigned int mbase = (unsigned)v1 | ((unsigned)(t + 1) << 16);
        unsigned long long off = 0;
        while (true) {
          const bool has = bany(ext);
          const unsigned long long mask = wave_ballot(has);
          if (!mask) break;
          if (has) {
            const int v = bpop_lowest(ext);
            const unsigned long long i = top + off + lanes_below(mask);
#pragma unroll
            for (int w = 0; w < W; ++w) stX[w * cap + i] = Xn.w[w];
            if (ENUM) {
              const Bits<W> Sn = bor(S, bsingle<W>(v));
#pragma unroll
              for (int w = 0; w < W; ++w) stS[w * cap + i] = Sn.w[w];
            }
            stM[i] = mbase | ((unsigned)v << 8);
          }
          off += __popcll(mask);
        }
        top += tot;
      }
    }

    // ---- donate the oldest chunk when other wavefronts are idle
    ++steps;
    if ((steps % (unsigned long long)wk.donate_check) == 0 && top - bot >= 2 * CC_CHUNK) {
      int idle = 0;
      if (lane == 0) idle = ld_acquire(&ctl->idle);
      idle = __shfl(idle, 0, CC_WAVE);
      if (idle > 0) {
        long long pos = -1;
        if (lane == 0) pos = q_reserve_push(ctl, wk);
        pos = bcast_i64(pos);
        if (pos >= 0) {
          const unsigned long long cell = (unsigned long long)pos & (wk.qcap - 1);
          const unsigned long long i = bot + lane;
#pragma unroll
          for (int w = 0; w < W; ++w) wk.qX[(cell * W + w) * CC_CHUNK + lane] = stX[w * cap + i];
          if (ENUM) {
#pragma unroll
            for (int w = 0; w < W; ++w) wk.qS[(cell * W + w) * CC_CHUNK + lane] = stS[w * cap + i];
          }
          wk.qM[cell * CC_CHUNK + lane] = stM[i];
          if (lane == 0) wk.qN[cell] = CC_CHUNK;
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
          if (lane == 0) st_release(&wk.qseq[cell], (unsigned long long)pos + 1ull);
          bot += CC_CHUNK;
          ++donated;
        }
      }
    }
  }

  if (lane == 0) {
    atomicAdd(&ctl->dfs_batches, batches);
    if (donated) atomicAdd(&ctl->donations, donated);
  }
  __syncthreads();
  for (int i = tid; i < CC_HSLOTS; i += CC_BLOCK) {
    if (hist_out && sHist[i]) atomicAdd(&hist_out[i], sHist[i]);
    if (count_front && sFront[i]) atomicAdd(&ctl->front[i], sFront[i]);
  }
}

// Resets the depth-first coordination state (and, for the writing pass of
// enumerate mode, computes where each cycle length starts in the output:
// lengths up to bfs_max_len were written by the breadth-first levels, longer
// ones come from the depth-first counting pass).  Does nothing when the
// breadth-first levels finished on their own.
__global__ void k_dfs_prepare(CcCtl *ctl, DfsWork wk0, DfsWork wk1, int n, int enum_bases) {
  if (ld_acquire(&ctl->mode) == 0) return;
  const DfsWork wk = (ctl->switch_level & 1) ? wk0 : wk1;
  for (unsigned long long i = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x;
       i < wk.qcap; i += (unsigned long long)gridDim.x * blockDim.x)
    wk.qseq[i] = i;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctl->root_cursor = 0;
    ctl->q_head = 0;
    ctl->q_tail = 0;
    ctl->busy = 0;
    ctl->idle = 0;
    if (enum_bases) {
      long long cb = 0, vb = 0;
      for (int k = 0; k <= n + 1 && k < CC_HSLOTS; ++k) {
        const long long c = (k <= ctl->bfs_max_len) ? (long long)ctl->hist[k]
                                                     : (long long)ctl->dfs_hist[k];
        ctl->len_cbase[k] = (unsigned long long)cb;
        ctl->len_vbase[k] = (unsigned long long)vb;
        ctl->len_cursor[k] = 0;
        cb += c;
        vb += c * k;
      }
    }
  }
}

// Enumerate mode: fold the depth-first counts into the histogram and close
// the offsets array with the total vertex count.
__global__ void k_finalize(CcCtl *ctl, OutDev out, int n) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  if (ld_acquire(&ctl->mode) != 0) {
    for (int k = ctl->bfs_max_len + 1; k <= n + 1 && k < CC_HSLOTS; ++k)
      ctl->hist[k] += ctl->dfs_hist[k];
  }
  long long c = 0, v = 0;
  for (int k = 0; k <= n && k < CC_HSLOTS; ++k) {
    c += (long long)ctl->hist[k];
    v += (long long)ctl->hist[k] * k;
  }
  if (c <= out.cyc_cap && v <= out.verts_cap && out.offs) out.offs[c] = v;
}

}  // namespace

// ------------------------------------------------------------------ launchers
hipError_t cc_launch_zero(void *p, size_t bytes, hipStream_t s) {
  const size_t words = bytes / 4;
  const int blocks = (int)min((size_t)1024, (words + 255) / 256 + 1);
  hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(256), 0, s, (unsigned int *)p, words);
  return hipGetLastError();
}

hipError_t cc_launch_ingest(int W, int n_graphs, const int *graph_vtx_off, int n_single,
                            const int *row_ptr, const int *col_idx, unsigned long long *adj,
                            int /*adj_stride_words*/, int *perm, int *label,
                            unsigned int *status, hipStream_t s) {
  if (W == 1)
    hipLaunchKernelGGL(k_ingest<1>, dim3(n_graphs), dim3(128), 0, s, graph_vtx_off, n_single,
                       row_ptr, col_idx, adj, perm, label, status);
  else
    hipLaunchKernelGGL(k_ingest<2>, dim3(n_graphs), dim3(128), 0, s, graph_vtx_off, n_single,
                       row_ptr, col_idx, adj, perm, label, status);
  return hipGetLastError();
}

hipError_t cc_launch_triplets(int W, bool en, GraphDev g, CcCtl *ctl, Frontier f3, OutDev out,
                              hipStream_t s) {
  if (W == 1) {
    if (en) hipLaunchKernelGGL((k_triplets<1, true>), dim3(1), dim3(CC_BLOCK), 0, s, g, ctl, f3, out);
    else hipLaunchKernelGGL((k_triplets<1, false>), dim3(1), dim3(CC_BLOCK), 0, s, g, ctl, f3, out);
  } else {
    if (en) hipLaunchKernelGGL((k_triplets<2, true>), dim3(1), dim3(CC_BLOCK), 0, s, g, ctl, f3, out);
    else hipLaunchKernelGGL((k_triplets<2, false>), dim3(1), dim3(CC_BLOCK), 0, s, g, ctl, f3, out);
  }
  return hipGetLastError();
}

hipError_t cc_launch_level(int W, bool en, GraphDev g, CcCtl *ctl, Frontier fin, Frontier fout,
                           OutDev out, int t, int forced_level, int blocks, hipStream_t s) {
  dim3 gr(blocks), bl(CC_BLOCK);
  if (W == 1) {
    if (en) hipLaunchKernelGGL((k_level<1, true>), gr, bl, 0, s, g, ctl, fin, fout, out, t, forced_level);
    else hipLaunchKernelGGL((k_level<1, false>), gr, bl, 0, s, g, ctl, fin, fout, out, t, forced_level);
  } else {
    if (en) hipLaunchKernelGGL((k_level<2, true>), gr, bl, 0, s, g, ctl, fin, fout, out, t, forced_level);
    else hipLaunchKernelGGL((k_level<2, false>), gr, bl, 0, s, g, ctl, fin, fout, out, t, forced_level);
  }
  return hipGetLastError();
}

hipError_t cc_launch_dfs(int W, bool en, GraphDev g, CcCtl *ctl, Frontier f0, Frontier f1,
                         DfsWork wk0, DfsWork wk1, OutDev out, unsigned long long *hist_out,
                         bool count_front, int blocks, unsigned long long idle_timeout,
                         hipStream_t s) {
  dim3 gr(blocks), bl(CC_BLOCK);
  const int cf = count_front ? 1 : 0;
  if (W == 1) {
    if (en) hipLaunchKernelGGL((k_dfs<1, true>), gr, bl, 0, s, g, ctl, f0, f1, wk0, wk1, out, hist_out, cf, idle_timeout);
    else hipLaunchKernelGGL((k_dfs<1, false>), gr, bl, 0, s, g, ctl, f0, f1, wk0, wk1, out, hist_out, cf, idle_timeout);
  } else {
    if (en) hipLaunchKernelGGL((k_dfs<2, true>), gr, bl, 0, s, g, ctl, f0, f1, wk0, wk1, out, hist_out, cf, idle_timeout);
    else hipLaunchKernelGGL((k_dfs<2, false>), gr, bl, 0, s, g, ctl, f0, f1, wk0, wk1, out, hist_out, cf, idle_timeout);
  }
  return hipGetLastError();
}

hipError_t cc_launch_dfs_prepare(CcCtl *ctl, DfsWork wk0, DfsWork wk1, int n, bool enum_bases,
                                 hipStream_t s) {
  hipLaunchKernelGGL(k_dfs_prepare, dim3(64), dim3(256), 0, s, ctl, wk0, wk1, n,
                     enum_bases ? 1 : 0);
  return hipGetLastError();
}

hipError_t cc_launch_finalize(CcCtl *ctl, OutDev out, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(64), 0, s, ctl, out, n);
  return hipGetLastError();
}
