// Internal declarations shared by the HIP kernels and the host runtime of
// libcc.  Not part of the public ABI (include/cc.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define CC_MAXN 1024
#define CC_HSLOTS (CC_MAXN + 2)   // per-length arrays: index 0..n+1
#define CC_ROWS(W) (64 * (W))     // vertices a W-word bitset graph can hold
#define CC_SLOTS(W) (CC_ROWS(W) + 2)  // per-length arrays of a W-word graph
// Graphs of more than 256 vertices (8 and 16 words): adjacency rows stay in
// device memory (their LDS copies would not fit) and end vertices take 16
// bits (the frontiers' end-vertex word is 32 bits wide).
#define CC_BIG(W) ((W) > 4)
#define CC_BATCH_MAXN 256         // largest graph of a batch (1, 2 or 4 words)
#define CC_WAVE 64
#define CC_BLOCK 256              // threads per block for the expansion kernels
#define CC_CHUNK 64               // paths per wavefront batch / donated chunk
#define CC_LEVEL_IPT 4            // paths per lane per chunk in the level kernel
#define CC_LEVEL_IPT_W4 3         // the same for four-word bitsets (n > 128)
#define CC_LEVEL_IPT_BIG 1        // and for eight and sixteen words (n > 256)
#define CC_DEC_WORDS 1280         // per-wavefront LDS words for decoded cycles (enumerate steps)
#define CC_HEAD_THREADS 1024      // threads of the one-block head kernel
// (256 for sixteen-word bitsets, so that a path's bitsets fit registers)
#define CC_HEAD_BLOCK(W) ((W) > 8 ? 256 : CC_HEAD_THREADS)
#define CC_ROOT_CLAIM 1024        // handed-over paths a depth-first wavefront claims at once
// Frontier and staged-cycle counters are split into CC_SHARDS shards, each
// on its own cache lines: a block appends to shard blockIdx % CC_SHARDS, so
// no counter sees more than 1/CC_SHARDS of the atomics (same-address
// device-scope atomics serialise across the chip).
#define CC_SHARDS 64

// Device-side error bits (CcCtl::status).
#define CC_DEV_NOT_SIMPLE 1u
#define CC_DEV_STACK_FULL 2u      // a depth-first stack had no room (results incomplete)
#define CC_DEV_IDLE_TIMEOUT 4u    // an idle wavefront gave up waiting (diagnostic only)
#define CC_DEV_CORRUPT 8u         // a depth-first consistency check failed (results discarded)
#define CC_DEV_LOST 16u           // a wavefront gave up on paths it was promised (results incomplete)
// First failed consistency check (CcCtl::diag): kind << 24 | low 24 bits of the value.
#define CC_DIAG_INBOX_COUNT 1u    // more paths announced than an inbox holds
#define CC_DIAG_REQUESTER 2u      // a work request names no wavefront of this launch
#define CC_DIAG_PATH 3u           // a path whose end vertices or length do not fit its graph
#define CC_DIAG_GRAPH 4u          // a path whose graph id is not in the batch

// skip bits for the paths handed to the depth-first kernel
#define CC_SKIP_FRONT 1           // their path count is already recorded
#define CC_SKIP_CLOSE 2           // their closures are already recorded

// State of one breadth-first step: it expands the paths with t vertices
// held in frontier buffer fbuf, by one level or by two, and decodes the
// cycles the previous step staged in stage pair spair (lengths slen0 and,
// after a two-level step, slen1; 0 = none).
struct StepState {
  int t;
  int fbuf;
  int spair;
  int slen0;
  int slen1;
  int prev_two;  // the previous step expanded two levels
  int done;      // the loop is over (nothing left, or handed over)
  int step;      // the step this state is for
};

// Control block of one run in device memory.  Zeroed by a kernel at the start
// of every run.  Per-shard arrays are shard-major, [s][k].
struct CcCtl {
  unsigned long long count_sh[CC_SHARDS][CC_HSLOTS];  // open paths with t vertices, per shard
  unsigned long long hist_sh[CC_SHARDS][CC_HSLOTS];   // cycles with k vertices, per shard
  // ---- zeroed in full before every run (the per-shard arrays above only in
  //      the columns 0..n+1 a run uses)
  unsigned long long cum_c[CC_HSLOTS];      // enumerate: cycles of length <= t (breadth-first)
  unsigned long long cum_v[CC_HSLOTS];      // enumerate: their vertex count
  unsigned long long dfs_hist[CC_HSLOTS];   // enumerate: depth-first part, counting pass
  unsigned long long len_cursor[CC_HSLOTS]; // enumerate: depth-first slot allocator per length
  unsigned long long len_cbase[CC_HSLOTS];  // enumerate: first cycle index of each length
  unsigned long long len_vbase[CC_HSLOTS];  // enumerate: first vertex offset of each length
  StepState ss[CC_HSLOTS];                  // step launch i reads ss[i]; its block 0 writes
                                            // ss[i + 1] (launch 0 is the head kernel)
  long long root_base[CC_MAXN];             // root range runs: index of the first stage-one
                                            // root of each vertex (by label)
  int orig_label[CC_MAXN];                  // root range runs: label of each original id
  // ---- read back by the host after every run (from here to the end)
  unsigned long long hist[CC_HSLOTS];       // final histogram (written by k_finalize)
  unsigned long long front[CC_HSLOTS];      // paths with t vertices expanded
  int launch_step[CC_HSLOTS];               // step of step launch i, plus one (0: loop over)
  int step_level[CC_HSLOTS];                // t of each step
  unsigned long long peak;                  // largest breadth-first frontier
  unsigned long long root_cursor;           // depth-first: next unclaimed handed-over path
  unsigned long long dfs_batches;           // depth-first batches processed (diagnostic)
  unsigned long long donations;             // chunks given away on request (diagnostic)
  unsigned long long dfs_lanes;             // depth-first: paths expanded over all steps (the
                                            // path total of a batch, which keeps no
                                            // per-length counts)
  unsigned long long dfs_idle_clk;          // depth-first: wavefront clocks spent without work
  unsigned long long dfs_wave_clk;          // depth-first: wavefront clocks from start to exit
  unsigned long long dfs_fills;             // depth-first: steps that popped from device memory
  unsigned long long dfs_spills;            // depth-first: ring entries moved to device memory
  unsigned long long dfs_gatomics;          // depth-first: global histogram atomics
  int levels_run;                           // breadth-first steps run
  int root_buf;                             // frontier buffer of the handed-over paths
  int mode;                                 // 0 = breadth-first, 1 = depth-first took over
  int switch_level;                         // path length handed to the depth-first kernel
  int skip;                                 // CC_SKIP_* bits for the handed-over paths
  int busy;                                 // depth-first wavefronts holding or seeking work
  unsigned int diag;                        // first failed consistency check, CC_DIAG_*
  unsigned int status;                      // CC_DEV_* bits
  int bfs_max_len;                          // longest cycle length final after the levels
  int head_steps;                           // steps run by the one-block head kernel
};

// Frontier of open paths, structure of arrays, CC_SHARDS shards of cap_s
// paths.  Path `off` of shard s is element i = s * cap_s + off; word w of its
// exclusion set X (label space) is X[w * cap + i]; likewise its vertex set S
// (original-id space, enumerate mode only); the end vertices (labels) are
// vv[i] = v1 | vt << 8, or vw[i] = v1 | vt << 16 beyond 256 vertices.
struct Frontier {
  unsigned long long *X;
  unsigned long long *S;
  unsigned short *vv;       // n <= 256
  unsigned int *vw;         // n > 256: v1 | vt << 16
  unsigned long long cap;    // CC_SHARDS * cap_s
  unsigned long long cap_s;
};

// Staged cycles of one level (enumerate mode): vertex-set bitsets in
// original-id space, sharded like a frontier: word w of cycle `off` of shard
// s is C[w * cap + s * cap_s + off].
struct Stage {
  unsigned long long *C;
  unsigned long long cap;
  unsigned long long cap_s;
};

// A range of stage-one roots: the (u, x, y) with l(u) < l(x) < l(y) and x, y
// neighbours of u, triangles included, numbered by u's original id, then
// x's, then y's; a run keeps the roots lo <= index < hi (all: 0, LLONG_MAX).
struct RootRange {
  long long lo = 0;
  long long hi = 0x7fffffffffffffffll;
};

// Relabelled graph: adjacency bitsets in label space (row l = neighbours of
// the vertex with label l), the same graph in original-id space, and
// perm[l] = original id of label l.
struct GraphDev {
  const unsigned long long *adj;
  const unsigned long long *adj_orig;
  const int *perm;
  int n;
};

// The breadth-first buffers of a run: two frontier buffers used in turn,
// and two pairs of staging buffers (one pair written by a step, the other
// decoded by it).
struct LevelBufs {
  Frontier f[2];
  Stage st[4];
};

// Enumeration output (cc_enumerate's buffers).  Only cycles with kmin <= k
// <= kmax are written; a cycle's global output index and vertex offset
// (over all lengths, ordered by length) are shifted down by cshift and
// vshift, the index and offset of the first cycle of length kmin.
struct OutDev {
  int *verts;
  long long *offs;
  long long verts_cap;
  long long cyc_cap;
  int kmin = 0;
  int kmax = 1 << 30;
  long long cshift = 0;
  long long vshift = 0;
  // Depth-first enumeration: the cycles the depth-first kernel finds (all
  // longer than bfs_max_len) are staged here as bitsets of original ids,
  // word w of the i-th of them (in output order) at dstage[w * dstage_cap +
  // i], and decoded by k_dfs_decode afterwards; those past dstage_cap, or
  // all of them when dstage is NULL, are written directly.
  unsigned long long *dstage = nullptr;
  long long dstage_cap = 0;
};

// Depth-first workspace: per-wavefront stacks, mailboxes and inboxes.  An
// entry is a frame: the open paths <q, v> for every v in E, sharing the
// exclusion set X, the first vertex v1 and the length t (and, enumerating,
// the original ids S of q).
// Mailbox words of wavefront w (its own 128-byte line):
//   mail[w * CC_MAIL + 0]  request: 0 none, r + 1 from wavefront r, CC_MAIL_CLOSED
//   mail[w * CC_MAIL + 1]  response to w's own request: 0 none, 1 work, 2 declined
//   mail[w * CC_MAIL + 2]  frames delivered into w's inbox
//   mail[w * CC_MAIL + 3]  frames w could give away (hint for victim choice)
#define CC_MAIL 32
#define CC_MAIL_CLOSED 0xffffffffu
struct DfsWork {
  unsigned long long *stackX;   // [nwaves][W][cap_w]
  unsigned long long *stackE;   // [nwaves][W][cap_w]
  unsigned long long *stackS;   // [nwaves][W][cap_w] (enumerate only)
  unsigned int *stackM;         // [nwaves][cap_w]: v1 | t<<16 (9 bits) | root<<31
  unsigned int *stackG;         // [nwaves][cap_w] graph id (batches only)
  unsigned long long cap_w;     // entries per wavefront stack
  unsigned int *mail;           // [nwaves][CC_MAIL]
  unsigned long long *inX;      // [nwaves][W][CC_CHUNK] inbox
  unsigned long long *inE;      // [nwaves][W][CC_CHUNK]
  unsigned long long *inS;      // [nwaves][W][CC_CHUNK] (enumerate only)
  unsigned int *inM;            // [nwaves][CC_CHUNK]
  unsigned int *inG;            // [nwaves][CC_CHUNK] (batches only)
  int nwaves;
  int donate_check;             // batches between mailbox checks
  int donate_min;               // paths a wavefront must hold before it gives some away
  int claim;                    // handed-over paths per claim; 0 = sized from the frontier
};

// A batch of graphs packed as one CSR (graph g owns vertices
// vtx_off[g] .. vtx_off[g+1]).  Its initial triplets sit in one array of
// root slots; graph g's slots are root_off[g] .. root_off[g+1] (an upper
// bound on its triplets), unused slots carry gid CC_NO_GRAPH.
#define CC_NO_GRAPH 0xffffffffu
struct BatchDev {
  const int *vtx_off;            // [G+1]
  const unsigned long long *adj; // label-space rows at (vtx_off[g] + l) * W
  const int *perm;               // perm[vtx_off[g] + l] = local id of label l
  const long long *root_off;     // [G+1]
  unsigned long long *rX;        // root slots: X words, word w at rX[w * rcap + i]
  unsigned short *rvv;           // root slots: v1 | vt << 8
  unsigned int *rgid;            // root slots: graph id or CC_NO_GRAPH
  unsigned long long rcap;
  unsigned long long r0, r1;     // slots handled by this launch
  unsigned long long *hist;      // per-graph histograms, graph g at hist[g * hist_stride]
  int hist_stride;
  int g0;                        // first graph of this launch (stage one)
  int n_graphs;                  // graphs in the batch (ids 0 .. n_graphs - 1)
};

// ------------------------------------------------------------------ launchers
// All return hipSuccess or the launch error.  `W` is 1, 2 or 4 (n <= 64, 128, 256).
hipError_t cc_launch_zero(void *p, size_t bytes, hipStream_t s);
// adj (label space) and adj_orig (original ids) rows are at (v0 + row) * W.
// bound (may be NULL) receives, per graph, sum over vertices of C(deg, 2):
// an upper bound on its initial triplets plus triangles.  reply (one graph
// only; may be NULL) is host-mapped memory that receives the status in
// word 1 and the bound in words 2..3, then 1 in word 0.
hipError_t cc_launch_ingest(int W, int n_graphs, const int *graph_vtx_off, int n_single,
                            const int *row_ptr, const int *col_idx, unsigned long long *adj,
                            unsigned long long *adj_orig, int *perm, int *label,
                            unsigned int *status, long long *bound, unsigned int *reply,
                            hipStream_t s);
// Stage one of graphs bt.g0 .. bt.g0 + n_graphs - 1 (one block each).
hipError_t cc_launch_triplets_batch(int W, BatchDev bt, int n_graphs, hipStream_t s);
// Stage one and the leading levels of the breadth-first loop on one block
// with the frontier in LDS (launch 0 for host_done), while a level's paths
// fit in lds_bytes of dynamic shared memory (two buffers); records the step
// the launches start at.
// With zero_ctl it first zeroes what a run on a graph of g.n vertices uses
// of the control block.  Only the stage-one roots in `roots` are kept.
hipError_t cc_launch_head(int W, bool enumerate, GraphDev g, CcCtl *ctl, const LevelBufs &b,
                          OutDev out, int forced_level, size_t lds_bytes,
                          unsigned int *host_done, bool zero_ctl, RootRange roots,
                          hipStream_t s);
// out (device) receives the number of stage-one roots of graph g.
hipError_t cc_launch_root_total(int W, GraphDev g, long long *out, hipStream_t s);
int cc_head_capacity(int W, bool enumerate, size_t lds_bytes);
size_t cc_head_static_lds(int W, bool enumerate);
// Launch `launch` (>= 1) of the breadth-first loop: one step on `blocks`
// blocks, the one recorded by the previous launch.  host_done (pinned host
// memory, may be NULL): host_done[0] receives launch + 1 once the loop is
// over (nothing left, or handed over to the depth-first kernel; then
// host_done[2] = 1 first), host_done[1] launch + 1 when the launch starts,
// so the host can stop launching and keep only a few queued.
hipError_t cc_launch_step(int W, bool enumerate, GraphDev g, CcCtl *ctl, const LevelBufs &b,
                          OutDev out, int launch, int forced_level, int max_children, bool two,
                          int blocks, unsigned int *host_done, hipStream_t s);
// Blocks of the step kernel resident per CU (its grid is that many per CU).
int cc_step_blocks_per_cu(int W, bool enumerate);
// The handed-over paths are in frontier f0 or f1 (CcCtl::root_buf); the
// workspace wk has memory of its own.  Cycle counts
// of block b go to hist_out[(b % CC_SHARDS) * hist_stride + k] (hist_out
// NULL: not counted).
hipError_t cc_launch_dfs(int W, bool enumerate, GraphDev g, CcCtl *ctl, Frontier f0,
                         Frontier f1, DfsWork wk, OutDev out,
                         unsigned long long *hist_out, int hist_stride, bool count_front,
                         int blocks, unsigned long long idle_timeout, hipStream_t s);
// Blocks of the depth-first kernel resident per CU (its LDS ring and rows
// set this); a persistent grid larger than cus times this would have blocks
// that start only after others have left.
int cc_dfs_blocks_per_cu(int W, bool en, bool batch);
// Batched depth-first run over the root slots bt.r0 .. bt.r1 (workspace wk).
hipError_t cc_launch_dfs_batch(int W, GraphDev g, CcCtl *ctl, DfsWork wk, BatchDev bt,
                               int blocks, unsigned long long idle_timeout, hipStream_t s);
// Zeroes wk's mailboxes and the claim and busy counters (always), and with
// enum_bases computes the output base of each cycle length.
hipError_t cc_launch_dfs_decode(int W, GraphDev g, const CcCtl *ctl, OutDev out, int blocks,
                                hipStream_t s);
hipError_t cc_launch_dfs_prepare(CcCtl *ctl, DfsWork wk, int n, bool enum_bases, hipStream_t s);
hipError_t cc_launch_finalize(CcCtl *ctl, OutDev out, int n, bool enumerate, hipStream_t s);
// After a complete enumerate run: the cycles of each length in out into
// ascending lexicographic order (tmp: room for the output's vertex ids; ia,
// ib: room for its cycle count each).  A no-op when the output did not fit.
// The cycles of a finished enumeration (verts_old/offs_old, nc of them)
// regrouped by stage-one root into verts_new/offs_new (offs_new: nc + 1
// entries), and first[r] = index of root r's first cycle, first[R] = nc
// unless a cycle was malformed.  work: cc_group_roots_workspace(nc) bytes.
size_t cc_group_roots_workspace(long long nc);
hipError_t cc_launch_group_roots(int W, GraphDev g, const int *label, const int *verts_old,
                                 const long long *offs_old, long long nc, long long R,
                                 int *verts_new, long long *offs_new, long long *first, void *work,
                                 hipStream_t s);
hipError_t cc_launch_sort_cycles(const CcCtl *ctl, OutDev out, int n, int *tmp, unsigned *ia,
                                 unsigned *ib, hipStream_t s);
