// Internal declarations shared by the HIP kernels and the host runtime of
// libcc.  Not part of the public ABI (include/cc.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define CC_MAXN 128
#define CC_HSLOTS (CC_MAXN + 2)   // histogram / per-length arrays: index 0..n+1
#define CC_WAVE 64
#define CC_BLOCK 256              // threads per block for the expansion kernels
#define CC_CHUNK 64               // paths per wavefront batch / donated chunk

// Device-side error bits (CcCtl::status).
#define CC_DEV_NOT_SIMPLE 1u
#define CC_DEV_STACK_FULL 2u      // depth-first stack and donation queue both full
#define CC_DEV_IDLE_TIMEOUT 4u    // an idle wavefront gave up waiting (diagnostic only)

// Control block of one run in device memory.  Zeroed by a kernel at the start
// of every run.  All counters are 64-bit.
struct CcCtl {
  unsigned long long count[CC_HSLOTS];     // count[t]: open paths with t vertices written
  unsigned long long hist[CC_HSLOTS];      // hist[k]: cycles with k vertices
  unsigned long long front[CC_HSLOTS];     // front[t]: paths with t vertices expanded
  unsigned long long dfs_hist[CC_HSLOTS];  // enumerate: depth-first part, counting pass
  unsigned long long len_cursor[CC_HSLOTS];// enumerate: depth-first slot allocator per length
  unsigned long long len_cbase[CC_HSLOTS]; // enumerate: first cycle index of each length
  unsigned long long len_vbase[CC_HSLOTS]; // enumerate: first vertex offset of each length
  unsigned long long peak;                 // largest breadth-first frontier
  unsigned long long root_cursor;          // depth-first: next unclaimed root path
  unsigned long long q_head, q_tail;       // depth-first donation queue positions
  unsigned long long dfs_batches;          // depth-first batches processed (diagnostic)
  unsigned long long donations;            // chunks donated (diagnostic)
  int mode;                                // 0 = breadth-first, 1 = depth-first took over
  int switch_level;                        // path length handed to the depth-first kernel
  int skip_first;                          // 1: the roots' first expansion was already counted
  int busy;                                // depth-first wavefronts holding or seeking work
  int idle;                                // depth-first wavefronts waiting for work
  unsigned int status;                     // CC_DEV_* bits
  int bfs_max_len;                         // longest cycle written by the breadth-first part
  int pad;
};

// Frontier of open paths, structure of arrays, capacity `cap` paths.
// Word w of path i's exclusion set X is X[w * cap + i]; likewise S (vertex
// set, enumerate mode only); vv[i] = v1 | vt << 8 (ids are labels).
struct Frontier {
  unsigned long long *X;
  unsigned long long *S;
  unsigned short *vv;
  unsigned long long cap;
};

// Relabelled graph: adjacency bitsets in label space (row l = neighbours of
// the vertex with label l, W words per row) and perm[l] = original id.
struct GraphDev {
  const unsigned long long *adj;
  const int *perm;
  int n;
};

// Enumeration output (cc_enumerate's buffers).
struct OutDev {
  int *verts;
  long long *offs;
  long long verts_cap;
  long long cyc_cap;
};

// Depth-first workspace: per-wavefront stacks and the donation queue.
struct DfsWork {
  unsigned long long *stackX;   // [nwaves][W][cap_w]
  unsigned long long *stackS;   // [nwaves][W][cap_w] (enumerate only)
  unsigned int *stackM;         // [nwaves][cap_w]: v1 | vt<<8 | t<<16 | root<<24
  unsigned long long cap_w;     // items per wavefront stack
  unsigned long long *qseq;     // [qcap] cell sequence numbers
  unsigned long long *qX;       // [qcap][W][CC_CHUNK]
  unsigned long long *qS;       // [qcap][W][CC_CHUNK]
  unsigned int *qM;             // [qcap][CC_CHUNK]
  unsigned int *qN;             // [qcap] items in the cell
  unsigned long long qcap;
  int max_children;             // upper bound on extensions of one path
  int donate_check;             // batches between donation checks
};

// ------------------------------------------------------------------ launchers
// All return hipSuccess or the launch error.  `W` is 1 (n <= 64) or 2.
hipError_t cc_launch_zero(void *p, size_t bytes, hipStream_t s);
hipError_t cc_launch_ingest(int W, int n_graphs, const int *graph_vtx_off, int n_single,
                            const int *row_ptr, const int *col_idx, unsigned long long *adj,
                            int adj_stride_words, int *perm, int *label, unsigned int *status,
                            hipStream_t s);
hipError_t cc_launch_triplets(int W, bool enumerate, GraphDev g, CcCtl *ctl, Frontier f3,
                              OutDev out, hipStream_t s);
hipError_t cc_launch_level(int W, bool enumerate, GraphDev g, CcCtl *ctl, Frontier fin,
                           Frontier fout, OutDev out, int t, int forced_level, int blocks,
                           hipStream_t s);
// The depth-first workspace lives in the frontier buffer that does not hold
// the handed-over paths: wk0 is carved from buffer 0, wk1 from buffer 1.
hipError_t cc_launch_dfs(int W, bool enumerate, GraphDev g, CcCtl *ctl, Frontier f0,
                         Frontier f1, DfsWork wk0, DfsWork wk1, OutDev out,
                         unsigned long long *hist_out, bool count_front, int blocks,
                         unsigned long long idle_timeout, hipStream_t s);
hipError_t cc_launch_dfs_prepare(CcCtl *ctl, DfsWork wk0, DfsWork wk1, int n, bool enum_bases,
                                 hipStream_t s);
hipError_t cc_launch_finalize(CcCtl *ctl, OutDev out, int n, hipStream_t s);
