/*
 * cc.h -- C ABI of libcc: enumeration of all chordless cycles of a finite
 * undirected simple graph on an MI355X (gfx950) GPU.
 *
 * A chordless cycle is an induced subgraph that is a cycle (Section 1 of
 * Jradi et al., "A GPU-based parallel algorithm for enumerating all
 * chordless cycles in graphs").  The library finds every such cycle exactly
 * once with the paper's method: a degree labelling of the vertices
 * (Section 2), the initial triplets and the triangles (Section 4.3,
 * Algorithm 2), then one-vertex extension of every open chordless path with
 * a chord test (Section 4.4, Algorithm 3), level by level (Algorithm 4).
 * When a level's frontier would exceed the caller's memory budget the
 * remaining work continues depth-first on per-wavefront stacks.
 *
 * Conventions for every entry point:
 *  - Graphs are int32 CSR: row_ptr[n+1] (row_ptr[0] = 0, non-decreasing),
 *    col_idx[row_ptr[n]]; each undirected edge appears in both lists.  Lists
 *    need not be sorted.  The graph must be simple: no self-loop, no
 *    repeated neighbour, symmetric, ids in [0, n).  1 <= n <= CC_MAX_VERTICES
 *    (n = 0 is accepted and has no cycles).
 *  - The "length" of a cycle is its number of vertices k (3 <= k <= n).
 *  - Cycles are reported in canonical form: starting at the vertex with the
 *    smallest original id, continuing towards the smaller of that vertex's
 *    two cycle neighbours.  Enumeration output is ordered by length; the
 *    order among cycles of equal length is unspecified unless CC_SORTED is
 *    set (then it is ascending lexicographic order of the vertex lists).
 *  - Pointers are host pointers unless a CC_*_DEVICE flag says otherwise.
 *    Device pointers must be device-accessible memory of the current HIP
 *    device.  All GPU work is ordered on cc_options.stream; every call
 *    returns only after its results are complete (the call synchronises
 *    that stream).
 *  - The caller owns every buffer it passes; the library owns a handle from
 *    the call that creates it until the matching release call.  A handle
 *    must not be used from two threads at once; separate handles may run
 *    concurrently on separate streams.
 *  - Errors are returned as cc_status; outputs are unspecified after an
 *    error unless stated otherwise.
 */
#ifndef CC_H
#define CC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CC_MAX_VERTICES 1024       /* one graph (cc_prepare); beyond 256 vertices the
                                      adjacency rows are read from device memory and
                                      every breadth-first level runs on the full grid */
#define CC_MAX_BATCH_VERTICES 256  /* each graph of a batch or of a serving request */
#define CC_ABI_VERSION 2

typedef enum cc_status {
  CC_OK = 0,
  CC_ERR_INVALID_ARG = -1,      /* null pointer, negative size, bad flags     */
  CC_ERR_NOT_SIMPLE = -2,       /* self-loop, repeated or one-way edge, bad id */
  CC_ERR_TOO_LARGE = -3,        /* n > CC_MAX_VERTICES                         */
  CC_ERR_BUFFER_TOO_SMALL = -4, /* output buffer too small; sizes reported     */
  CC_ERR_OUT_OF_MEMORY = -5,    /* device allocation failed / budget too small */
  CC_ERR_DEVICE = -6,           /* HIP runtime error or device-side failure    */
  CC_ERR_NO_DEVICE = -7,        /* no usable gfx950 device                     */
  CC_ERR_NOT_READY = -8,        /* serving: the request has not finished yet    */
  CC_ERR_INTERNAL = -9          /* a device-side consistency check failed; the
                                   results of the call are discarded (see
                                   cc_run_info.device_diag)                     */
} cc_status;

/* cc_options.flags */
#define CC_INPUT_DEVICE  (1u << 0) /* row_ptr/col_idx (and batch offsets) are device pointers */
#define CC_OUTPUT_DEVICE (1u << 1) /* cc_enumerate's verts/offsets are device pointers        */
#define CC_FORCE_DFS     (1u << 2) /* take the depth-first path from level dfs_level on      */
#define CC_PROFILE       (1u << 3) /* time each kernel of a run with HIP events (cc_run_info) */
/* (1u << 4) is not used */
#define CC_ONE_LEVEL_STEPS (1u << 5)  /* expand one level per breadth-first step, never two
                                        (same results)                                     */
#define CC_SORTED        (1u << 6) /* cc_enumerate / cc_enumerate_lengths: the cycles of each
                                      length in ascending lexicographic order of their
                                      canonical vertex lists, so the whole output is sorted
                                      by (k, c0, c1, ...) (Algorithm 1's output set C in one
                                      fixed order); sorted on the device after the run    */

typedef struct cc_options {
  void *stream;                  /* hipStream_t; NULL = the null stream                 */
  int64_t frontier_budget_bytes; /* device memory for open paths; 0 = 4 GiB             */
  uint32_t flags;                /* CC_* flags above                                     */
  int32_t dfs_level;             /* with CC_FORCE_DFS: path length t >= 3 whose frontier
                                    is handed to the depth-first kernel                  */
  int32_t dfs_waves_per_cu;      /* depth-first kernel occupancy; 0 = default (24)       */
  int32_t bfs_blocks;            /* grid of the level kernel; 0 = one resident wave of
                                    blocks (occupancy query, at most 6 per CU)          */
  int32_t dfs_donate_min;        /* depth-first: a wavefront donates work to idle ones once
                                    it holds at least this many paths; 0 = default      */
  int32_t dfs_claim;             /* depth-first: handed-over paths claimed per atomic
                                    (multiple of 64); 0 = sized from the frontier       */
} cc_options;

typedef struct cc_graph cc_graph;

/* Statistics of the most recent count/histogram/enumerate call on a handle. */
typedef struct cc_run_info {
  int64_t cycles;            /* total chordless cycles                               */
  int64_t paths;             /* open chordless paths expanded (sum over lengths)     */
  int64_t peak_frontier;     /* largest level frontier held in breadth-first mode     */
  int32_t switch_level;      /* path length handed to the depth-first kernel, 0=none */
  int32_t levels_launched;   /* full-grid breadth-first step launches             */
  double gpu_ms;             /* device time of the call, HIP events around its work  */
  /* With CC_PROFILE only (else 0): device time of each part of the run.       */
  double stage1_ms;          /* initial triplets and triangles                       */
  double level_ms;           /* the full-grid breadth-first step launches            */
  double dfs_ms;             /* depth-first kernels and their preparation            */
  int64_t level_bytes;       /* frontier and output bytes those launches must move    */
  int64_t device_diag;       /* after CC_ERR_INTERNAL: which check failed (kind << 24 |
                                low 24 bits of the offending value), else 0          */
  int32_t head_steps;        /* leading small steps run on one block before the
                                full-grid launches                                   */
  int32_t reserved;
  double head_ms;            /* CC_PROFILE: device time of those leading steps       */
  int64_t head_bytes;        /* CC_PROFILE: bytes those leading steps must move      */
  int64_t dfs_steps;         /* depth-first kernel: wavefront steps (up to 64 paths
                                each) run over the call                              */
  int64_t dfs_donations;     /* depth-first kernel: chunks of work handed to idle
                                wavefronts                                           */
  double dfs_lane_use;       /* depth-first kernel: paths expanded / (64 * steps)    */
  double dfs_idle_frac;      /* depth-first kernel: share of wavefront time spent
                                looking for work                                     */
  int64_t dfs_fills;         /* depth-first kernel: steps whose frames came back from
                                device memory (the LDS part of the stack was empty)  */
  int64_t dfs_spills;        /* depth-first kernel: stack entries moved from LDS to
                                device memory                                        */
  int64_t dfs_global_adds;   /* depth-first kernel (batches): histogram additions in
                                device memory                                        */
} cc_run_info;

/*
 * cc_prepare -- validate a graph and compute its degree labelling
 * (Section 2: repeatedly remove a vertex of minimum remaining degree; the
 * i-th removed vertex gets label i, 0-based; ties go to the smallest id).
 *   n        number of vertices, 0 <= n <= CC_MAX_VERTICES
 *   row_ptr  n+1 offsets; col_idx row_ptr[n] neighbour ids (host, or device
 *            with CC_INPUT_DEVICE).  With CC_INPUT_DEVICE, col_idx must hold
 *            row_ptr[n] entries whenever row_ptr[n] <= n*(n-1).
 *   opt      may be NULL (defaults).  The options are kept in the handle.
 *   out      receives the handle; the inputs may be freed when this returns.
 * Errors: INVALID_ARG, TOO_LARGE, NOT_SIMPLE (Section 2 assumes a simple
 * graph), OUT_OF_MEMORY, DEVICE, NO_DEVICE.  *out is NULL on error.
 */
cc_status cc_prepare(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                     const cc_options *opt, cc_graph **out);

/* cc_count -- total number of chordless cycles, triangles included (the
 * paper's C3 + #clc, Table 1).  Runs the count-only pipeline. */
cc_status cc_count(cc_graph *g, int64_t *total);

/* cc_histogram -- hist[k] = number of chordless cycles with k vertices for
 * 0 <= k < hist_len (entries 0..2 are zero); hist_len >= n+1 (host array).
 * Count-only: no cycle is stored (the paper's count-only mode, Table 1
 * footnote on Grid 8x10). */
cc_status cc_histogram(cc_graph *g, int64_t *hist, int32_t hist_len);

/*
 * cc_enumerate -- write every chordless cycle (Algorithm 1's output set C).
 *   verts[verts_cap]        concatenated cycles, original vertex ids
 *   offsets[cycles_cap + 1] cycle i is verts[offsets[i] .. offsets[i+1])
 *   n_cycles, n_verts       receive the exact totals (host int64)
 * Both buffers are host memory, or device memory with CC_OUTPUT_DEVICE.
 * Sizing: the totals equal sum(hist) and sum(k * hist[k]) from
 * cc_histogram.  If cycles_cap < total cycles or verts_cap < total
 * vertices, returns CC_ERR_BUFFER_TOO_SMALL with *n_cycles / *n_verts set
 * to the required sizes; buffer contents are then unspecified.
 */
cc_status cc_enumerate(cc_graph *g, int32_t *verts, int64_t verts_cap, int64_t *offsets,
                       int64_t cycles_cap, int64_t *n_cycles, int64_t *n_verts);

/*
 * cc_enumerate_lengths -- write the chordless cycles with k_min <= k <= k_max
 * vertices only: the slice of cc_enumerate's output that holds those
 * lengths, with offsets starting at 0.  A caller whose buffers cannot hold
 * every cycle pages through the output one range of lengths at a time
 * (Section 6 names larger outputs than device memory holds as future work;
 * the unit of a page here is one cycle length, since the order of cycles of
 * equal length is unspecified).  Each call runs the enumeration again;
 * cycles outside the range are found but not written.
 *   k_min, k_max            0 <= k_min <= k_max
 *   verts, offsets, caps    as cc_enumerate, for the range only
 *   n_cycles, n_verts       receive the range's exact totals
 * The range's sizes come from the histogram (from the handle's last
 * complete call, else a counting run first).  If a buffer is too small,
 * returns CC_ERR_BUFFER_TOO_SMALL with the required sizes and writes
 * nothing.  Errors otherwise as cc_enumerate.
 */
cc_status cc_enumerate_lengths(cc_graph *g, int32_t k_min, int32_t k_max, int32_t *verts,
                               int64_t verts_cap, int64_t *offsets, int64_t cycles_cap,
                               int64_t *n_cycles, int64_t *n_verts);

/*
 * Stage-one roots.  Every chordless cycle is found from exactly one root:
 * its canonical triplet <x, u, y> (Section 2: u the cycle's lowest label, x
 * and y its neighbours on the cycle, l(x) < l(y)), or the triangle it is.
 * The roots of a graph are the (u, x, y) with x, y neighbours of u and
 * l(u) < l(x) < l(y), triangles included, numbered 0 .. total-1 in the order
 * of u's original id, then x's, then y's.  A range of roots therefore
 * selects a fixed part of the cycle set, and consecutive ranges partition
 * it: an output larger than a caller's buffers (Section 6 names larger
 * outputs as future work) is paged by ranges of roots, each page costing
 * only the search below its own roots, and a page may split a length.
 */
/* cc_root_total -- *n_roots = number of stage-one roots. */
cc_status cc_root_total(cc_graph *g, int64_t *n_roots);

/* cc_histogram_roots -- as cc_histogram, for the cycles found from roots
 * root_lo <= index < root_hi only (0 <= root_lo <= root_hi). */
cc_status cc_histogram_roots(cc_graph *g, int64_t root_lo, int64_t root_hi, int64_t *hist,
                             int32_t hist_len);

/* cc_enumerate_roots -- as cc_enumerate, for the cycles found from roots
 * root_lo <= index < root_hi only: ordered by length, offsets from 0,
 * sizes from cc_histogram_roots of the same range; BUFFER_TOO_SMALL reports
 * the range's sizes.  CC_SORTED sorts each length of the page. */
cc_status cc_enumerate_roots(cc_graph *g, int64_t root_lo, int64_t root_hi, int32_t *verts,
                             int64_t verts_cap, int64_t *offsets, int64_t cycles_cap,
                             int64_t *n_cycles, int64_t *n_verts);

/* cc_enumerate_by_roots -- the whole output of cc_enumerate, in one run,
 * with the cycles grouped by stage-one root (roots in the order above;
 * within a root, by length).  root_first[r] is the index of root r's first
 * cycle (roots without cycles get the next root's), root_first[R] = the
 * number of cycles, R = cc_root_total; so the cycles of roots lo .. hi-1
 * are cycles root_first[lo] .. root_first[hi]-1, one contiguous piece of
 * the output, the same cycle set as cc_enumerate_roots(lo, hi).  This is
 * how a large output is paged when it fits device memory twice over: one
 * search, then pages by root ranges copied out of it.
 *   verts, offsets          as cc_enumerate (offsets[n_cycles] = n_verts)
 *   root_first, roots_cap   R + 1 int64 entries (roots_cap >= R + 1, else
 *                           CC_ERR_INVALID_ARG)
 * Device or host pointers per CC_OUTPUT_DEVICE.  The run works in device
 * memory of its own: staging of the caller's capacities plus about 16
 * bytes per cycle (and, for host output, the output's size again).  If a
 * buffer is too small, returns CC_ERR_BUFFER_TOO_SMALL with the required
 * sizes after the run; CC_ERR_INTERNAL if a cycle had no root.  CC_SORTED
 * is ignored (the order within a root is by length only). */
cc_status cc_enumerate_by_roots(cc_graph *g, int32_t *verts, int64_t verts_cap, int64_t *offsets,
                                int64_t cycles_cap, int64_t *root_first, int64_t roots_cap,
                                int64_t *n_cycles, int64_t *n_verts);

/* cc_labels -- labels[v] = degree label of vertex v (host array of n). */
cc_status cc_labels(cc_graph *g, int32_t *labels);

/* cc_frontier -- front[t] = number of open chordless paths with t vertices
 * that the last run expanded (front[3] = |T(G)|, Section 2), for
 * 0 <= t < len, len >= n+1 (host array). */
cc_status cc_frontier(cc_graph *g, int64_t *front, int32_t len);

/* cc_level_times -- device time in ms of each breadth-first level kernel
 * of the last call made with CC_PROFILE: ms[t] for the level that expands
 * paths with t vertices (0 where no level was launched), 0 <= t < len,
 * len >= n+1 (host array).  All zeros after a call without CC_PROFILE. */
cc_status cc_level_times(cc_graph *g, double *ms, int32_t len);

/* cc_last_run -- statistics of the last count/histogram/enumerate call. */
cc_status cc_last_run(cc_graph *g, cc_run_info *info);

/* cc_release -- free a handle and its device memory (NULL is ignored). */
void cc_release(cc_graph *g);

/*
 * cc_histogram_noalloc -- cc_prepare + cc_histogram + cc_release in one call
 * that allocates nothing, for callers that cannot allocate (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Every buffer beyond the caller's inputs and output lives in one fixed
 * device array inside the library (64 MiB per GPU, held from the library's
 * load until the process ends; 24 MiB of it for the breadth-first
 * frontiers, the rest for the depth-first stacks).
 *   n        number of vertices, 0 <= n <= CC_MAX_VERTICES
 *   row_ptr, col_idx  the graph as int32 CSR in DEVICE memory (as
 *            cc_prepare with CC_INPUT_DEVICE)
 *   hist     DEVICE array of hist_len >= n+1 int64: hist[k] = chordless
 *            cycles with k vertices (as cc_histogram), zeros past n
 *   stream   hipStream_t the work is ordered on (NULL: the null stream); the
 *            call returns after its results are complete
 * Errors: INVALID_ARG, TOO_LARGE (n > CC_MAX_VERTICES), NOT_SIMPLE,
 * OUT_OF_MEMORY (the graph's initial triplets, or its depth-first stacks,
 * need more than the fixed array holds), INTERNAL, DEVICE, NO_DEVICE.
 * Calls that overlap on one GPU share its array and race: serialise them.
 */
cc_status cc_histogram_noalloc(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                               int64_t *hist, int32_t hist_len, void *stream);

/* ------------------------------------------------------------- batches
 * Many small graphs enumerated together (count-only).  The graphs are packed
 * as one CSR: graph g owns vertices graph_vtx_off[g] .. graph_vtx_off[g+1]
 * (global ids in row_ptr/col_idx), graph_vtx_off[0] = 0, every graph has at
 * most CC_MAX_BATCH_VERTICES vertices and no edge leaves its graph.
 */
typedef struct cc_batch cc_batch;

#define CC_BATCH_PERSISTENT 0 /* stage one of all graphs in one launch, then one
                                 persistent depth-first launch with work stealing
                                 over every graph's initial triplets             */
#define CC_BATCH_PER_GRAPH  1 /* the same kernels launched once per graph, the
                                 depth-first kernel on the same full grid
                                 (the baseline the persistent form is compared to) */

/* cc_prepare_batch -- validate every graph and compute its degree labelling
 * (one block per graph).  graph_vtx_off has n_graphs+1 entries; with
 * CC_INPUT_DEVICE all three arrays are device pointers.  Errors as
 * cc_prepare (NOT_SIMPLE if any graph is not simple).  The batch has a
 * handle type of its own (cc_batch, not cc_graph) so that single-graph calls
 * cannot be given a batch by mistake. */
cc_status cc_prepare_batch(int32_t n_graphs, const int32_t *graph_vtx_off, const int32_t *row_ptr,
                           const int32_t *col_idx, const cc_options *opt, cc_batch **out);

/* cc_histogram_batch -- per-graph histograms (Table 1's C3 and #clc columns
 * per length, for every graph of the batch), count-only, in the persistent
 * form.  Graph g with n_g vertices writes hists[hist_off[g] + k] = cycles
 * with k vertices, for 0 <= k <= n_g (n_g + 1 entries; entries 0..2 are 0).
 *   hists     host array the caller sizes to cover every graph's range
 *   hist_off  host array of n_graphs offsets, each >= 0; the ranges must not
 *             overlap (g * (max_n + 1) gives a dense [G x (max_n + 1)] table)
 * Errors: INVALID_ARG (NULL arrays with n_graphs > 0, a negative offset),
 * OUT_OF_MEMORY (workspace, or a depth-first stack ran out), INTERNAL, DEVICE.
 * The entries of hists outside the graphs' ranges are not touched. */
cc_status cc_histogram_batch(cc_batch *b, int64_t *hists, const int64_t *hist_off);

/* cc_histogram_batch_mode -- cc_histogram_batch with the launch form chosen:
 * mode is CC_BATCH_PERSISTENT (what cc_histogram_batch runs) or
 * CC_BATCH_PER_GRAPH; both give the same numbers. */
cc_status cc_histogram_batch_mode(cc_batch *b, int64_t *hists, const int64_t *hist_off,
                                  int32_t mode);

/* cc_batch_labels -- degree label of every vertex (host array of the total
 * vertex count, indexed by global id; labels are local to each graph). */
cc_status cc_batch_labels(cc_batch *b, int32_t *labels);

/* cc_batch_last_run -- statistics of the last cc_histogram_batch call
 * (levels_launched counts kernel launches; paths is the batch total; with
 * CC_PROFILE in the batch's options, a persistent-form call also fills
 * stage1_ms and dfs_ms, HIP events on the batch's stream around stage one
 * and around the depth-first kernel). */
cc_status cc_batch_last_run(cc_batch *b, cc_run_info *info);

/* cc_release_batch -- free a batch handle (NULL is ignored). */
void cc_release_batch(cc_batch *b);

/* ------------------------------------------------------------- serving
 * A request loop for many independent graphs (count + histogram each).  A
 * dispatcher thread admits pending requests, in arrival order, into a free
 * device slot while the slot's capacities hold (graphs, vertices, adjacency
 * entries, and root slots: a graph needs sum over vertices of C(deg, 2)),
 * and runs each admitted group as one batch (stage one, then one persistent
 * depth-first launch on the slot's share of the CUs).  Slots run
 * concurrently, so requests that arrive while others are on the GPU start
 * as soon as a slot frees up.  Results do not depend on how requests were
 * grouped.
 */
typedef struct cc_server cc_server;

typedef struct cc_server_options {
  int32_t slots;             /* concurrent device slots; 0 = 4                       */
  int32_t max_batch_graphs;  /* graphs per batch; 0 = 256                            */
  int64_t slot_root_slots;   /* initial-triplet slots per batch; 0 = 4M               */
  int64_t slot_work_bytes;   /* depth-first workspace per slot; 0 = 256 MiB           */
  int32_t dfs_waves_per_cu;  /* wavefronts per CU shared by all slots; 0 = 16        */
  int32_t reserved;
} cc_server_options;

/* cc_server_create -- allocate the slots (device and pinned memory) and start
 * the dispatcher on the current HIP device. */
cc_status cc_server_create(const cc_server_options *opt, cc_server **out);

/* cc_server_submit -- queue one graph (host CSR, copied before returning);
 * *request_id receives its id.  Argument errors as cc_prepare; a graph
 * larger than a whole slot completes at once with CC_ERR_OUT_OF_MEMORY as
 * its request status. */
cc_status cc_server_submit(cc_server *sv, int32_t n, const int32_t *row_ptr,
                           const int32_t *col_idx, int64_t *request_id);

/* cc_server_result -- wait up to timeout_s for a request; on success write
 * its histogram (hist_len >= n+1), its latency from submission to
 * completion in ms, and its own status (CC_OK, CC_ERR_NOT_SIMPLE, ...), and
 * forget the request.  Returns CC_ERR_NOT_READY on timeout (the request
 * stays queryable). */
cc_status cc_server_result(cc_server *sv, int64_t request_id, double timeout_s, int64_t *hist,
                           int32_t hist_len, double *latency_ms, cc_status *request_status);

/* cc_server_stats -- stats[0] completed, [1] batches launched, [2] pending,
 * [3] rejected, [4] largest batch (len >= 5). */
cc_status cc_server_stats(cc_server *sv, int64_t *stats, int32_t len);

/* cc_server_destroy -- finish every queued request, stop, free (NULL ok). */
void cc_server_destroy(cc_server *sv);

/* cc_status_string -- static English description of a status code. */
const char *cc_status_string(cc_status s);

/* cc_abi_version -- CC_ABI_VERSION of the loaded library. */
int32_t cc_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* CC_H */
