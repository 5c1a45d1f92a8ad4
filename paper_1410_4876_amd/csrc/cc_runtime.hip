// Host runtime behind the C ABI of include/cc.h: validation of arguments,
// device memory, the level loop (Algorithm 4, without per-level readback),
// the hand-over to the depth-first kernel, and result readback.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstddef>
#include <chrono>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "cc.h"
#include "cc_internal.h"

static_assert(CC_BATCH_MAXN == CC_MAX_BATCH_VERTICES, "batch vertex limit");
static_assert(CC_MAXN == CC_MAX_VERTICES, "vertex limit");

namespace {

constexpr int64_t kDefaultBudget = 4ll << 30;
// Largest device staging for cc_enumerate into host buffers taken at the
// caller's capacities in one pass; larger capacities are sized exactly by a
// counting run first.
constexpr int64_t kHostStageBytes = 8ll << 30;
constexpr int kReplyWord = 8;       // ingest reply: words 8..11 of the pinned flag area
constexpr int kReplySpinUs = 2000;  // polling for it before a stream synchronisation
constexpr int kGroupWord = 12;      // cc_enumerate_by_roots check: words 12..13
static_assert(kReplyWord + 4 <= kGroupWord && kGroupWord + 2 <= 16,
              "the pinned flag area holds 16 words");
constexpr int kStepBlocksPerCu = 6;  // cap on the step grid per CU (7 ran 20 % slower)
constexpr int kLevelsAhead = 2;    // level launches queued beyond the device's progress
constexpr int kAheadWaitUs = 200;  // longest the host waits for that progress
constexpr double kIdleTimeoutSeconds = 30.0;

struct DeviceInfo {
  bool ok = false;
  int cus = 0;
  unsigned long long clock_hz = 0;
  size_t lds_block = 0;  // LDS a block may hold
};

std::mutex g_dev_mu;
DeviceInfo g_dev[64];

// Per-device set-up: checks the architecture, reads the CU count and the
// constant-rate clock, and keeps freed stream-ordered memory in the pool so
// per-call workspaces are cheap after the first call.
cc_status device_info(int dev, DeviceInfo *out) {
  if (dev < 0 || dev >= 64) return CC_ERR_NO_DEVICE;
  std::lock_guard<std::mutex> lk(g_dev_mu);
  if (!g_dev[dev].ok) {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) return CC_ERR_NO_DEVICE;
    if (std::strncmp(p.gcnArchName, "gfx950", 6) != 0) return CC_ERR_NO_DEVICE;
    int rate_khz = 0;
    if (hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess ||
        rate_khz <= 0)
      rate_khz = 100000;
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
      uint64_t thr = UINT64_MAX;
      (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    }
    // dynamic LDS for the head kernel's two frontier buffers: what a block
    // may hold, less the kernel's static part and a margin
    int lds = 0;
    (void)hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    g_dev[dev].lds_block = lds > 0 ? (size_t)lds : 0;
    g_dev[dev].cus = p.multiProcessorCount;
    g_dev[dev].clock_hz = (unsigned long long)rate_khz * 1000ull;
    g_dev[dev].ok = true;
  }
  *out = g_dev[dev];
  return CC_OK;
}

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Per-handle device/pinned resources are recycled through a small free list
// so that creating a handle per request (serving) costs no allocation after
// warm-up.
struct HandleRes {
  int device;
  void *d_blob;
  void *h_ctl;
  void *h_done;
  hipEvent_t ev0, ev1;
};
std::mutex g_pool_mu;
HandleRes g_pool[64];
int g_pool_n = 0;

bool pool_take(int device, HandleRes *r) {
  std::lock_guard<std::mutex> lk(g_pool_mu);
  for (int i = g_pool_n - 1; i >= 0; --i) {
    if (g_pool[i].device == device) {
      *r = g_pool[i];
      g_pool[i] = g_pool[--g_pool_n];
      return true;
    }
  }
  return false;
}

bool pool_give(const HandleRes &r) {
  std::lock_guard<std::mutex> lk(g_pool_mu);
  if (g_pool_n >= 64) return false;
  g_pool[g_pool_n++] = r;
  return true;
}

// Batches recycle theirs the same way: the device blob (graph data and
// control block), pinned staging for every host copy of a pass, the pinned
// control-block readback and the events.  A batch takes the smallest free
// set on its device that is large enough; a set that is too small is freed
// and a larger one allocated.
struct BatchRes {
  int device = -1;
  void *d_blob = nullptr;
  size_t blob_bytes = 0;
  char *h_stage = nullptr;
  size_t stage_bytes = 0;
  void *h_ctl = nullptr;
  hipEvent_t ev[6] = {};
};
std::mutex g_bpool_mu;
BatchRes g_bpool[16];
int g_bpool_n = 0;

void batch_res_free(BatchRes &r) {
  (void)hipSetDevice(r.device);
  if (r.d_blob) (void)hipFree(r.d_blob);
  if (r.h_stage) (void)hipHostFree(r.h_stage);
  if (r.h_ctl) (void)hipHostFree(r.h_ctl);
  for (hipEvent_t e : r.ev)
    if (e) (void)hipEventDestroy(e);
  r = BatchRes{};
}

// A set on `device` (the current device) with at least `stage` pinned
// bytes; its blob is grown later by batch_res_blob.
bool batch_res_take(int device, size_t stage, BatchRes *out) {
  BatchRes r;
  {
    std::lock_guard<std::mutex> lk(g_bpool_mu);
    int best = -1, any = -1;
    for (int i = 0; i < g_bpool_n; ++i) {
      if (g_bpool[i].device != device) continue;
      any = i;
      if (g_bpool[i].stage_bytes >= stage &&
          (best < 0 || g_bpool[i].stage_bytes < g_bpool[best].stage_bytes))
        best = i;
    }
    const int pick = best >= 0 ? best : any;
    if (pick >= 0) {
      r = g_bpool[pick];
      g_bpool[pick] = g_bpool[--g_bpool_n];
    }
  }
  r.device = device;
  bool ok = true;
  if (r.stage_bytes < stage) {
    if (r.h_stage) (void)hipHostFree(r.h_stage);
    r.h_stage = nullptr;
    r.stage_bytes = 0;
    ok = hipHostMalloc((void **)&r.h_stage, stage, hipHostMallocDefault) == hipSuccess;
    if (ok) r.stage_bytes = stage;
  }
  if (ok && !r.h_ctl) ok = hipHostMalloc(&r.h_ctl, sizeof(CcCtl), hipHostMallocDefault) == hipSuccess;
  for (hipEvent_t &e : r.ev)
    if (ok && !e) ok = hipEventCreate(&e) == hipSuccess;
  if (!ok) {
    batch_res_free(r);
    return false;
  }
  *out = r;
  return true;
}

// Grows the set's device blob to at least `bytes` (a device-wide
// synchronisation only when it grows).
bool batch_res_blob(BatchRes &r, size_t bytes) {
  if (r.blob_bytes >= bytes) return true;
  if (r.d_blob) (void)hipFree(r.d_blob);
  r.d_blob = nullptr;
  r.blob_bytes = 0;
  if (hipMalloc(&r.d_blob, bytes) != hipSuccess) return false;
  r.blob_bytes = bytes;
  return true;
}

void batch_res_give(BatchRes &r) {
  if (r.device < 0) return;
  {
    std::lock_guard<std::mutex> lk(g_bpool_mu);
    if (g_bpool_n < 16) {
      g_bpool[g_bpool_n++] = r;
      r = BatchRes{};
      return;
    }
  }
  batch_res_free(r);
}

}  // namespace

struct cc_graph {
  int device = 0;
  hipStream_t stream = nullptr;
  cc_options opt{};
  int32_t n = 0;
  int W = 1;
  int max_deg = 0;
  int64_t n_roots = -1;  // stage-one roots, once counted (a property of the graph)
  DeviceInfo dev{};
  void *d_blob = nullptr;  // adj | perm | label | status | ctl
  unsigned long long *d_adj = nullptr;       // label-space adjacency bitsets
  unsigned long long *d_adj_orig = nullptr;  // original-id adjacency bitsets
  int *d_perm = nullptr;
  int *d_label = nullptr;
  unsigned int *d_status = nullptr;
  CcCtl *d_ctl = nullptr;
  CcCtl *h_ctl = nullptr;  // pinned readback
  unsigned int *h_done = nullptr;  // pinned flag written by the level kernels
  unsigned int *d_done = nullptr;  // its device-side address
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  hipEvent_t evp[2 * CC_MAXN + 8] = {};  // CC_PROFILE: around each kernel group
  bool have_run = false;
  bool hist_ok = false;  // hist/front hold the results of a complete run
  int64_t pairs = 0;     // sum over vertices of C(deg, 2)
  int64_t hist[CC_HSLOTS]{};
  double level_ms[CC_HSLOTS]{};  // CC_PROFILE: per-level device time
  int64_t front[CC_HSLOTS]{};
  cc_run_info info{};
};

namespace {

cc_status hip_err(hipError_t e) {
  if (e == hipErrorOutOfMemory) return CC_ERR_OUT_OF_MEMORY;
  return e == hipSuccess ? CC_OK : CC_ERR_DEVICE;
}

#define CC_TRY(expr)                          \
  do {                                        \
    hipError_t e_ = (expr);                   \
    if (e_ != hipSuccess) return hip_err(e_); \
  } while (0)

// Address of a counter array inside the device-side control block.
unsigned long long *dev_field(CcCtl *ctl, size_t offset) {
  return (unsigned long long *)((char *)ctl + offset);
}

int64_t choose3(int64_t n) { return n < 3 ? 0 : n * (n - 1) * (n - 2) / 6; }

// 64-bit words per vertex bitset of a single graph of n vertices.
int words_for(int n) { return n <= 64 ? 1 : n <= 128 ? 2 : n <= 256 ? 4 : n <= 512 ? 8 : 16; }

// Bytes of a frontier path's end-vertex word: two up to 256 vertices, four
// beyond.
size_t vv_bytes(int W) { return W > 4 ? 4 : 2; }

// The head kernel's dynamic LDS for its in-LDS frontier: what a block may
// hold, less the kernel's static part and a margin.
size_t head_dyn_lds(int W, bool en, size_t lds_block) {
  const size_t stat = cc_head_static_lds(W, en) + 4096;
  return lds_block > stat ? lds_block - stat : 0;
}

// Carves one sharded frontier buffer (SoA: X words, S words, end vertices)
// of CC_SHARDS * cap_s paths out of `base`.
Frontier carve_frontier(char *base, unsigned long long cap_s, int W, bool en) {
  Frontier f{};
  const unsigned long long cap = cap_s * CC_SHARDS;
  size_t off = 0;
  f.X = (unsigned long long *)(base + off);
  off = align_up(off + cap * W * 8, 256);
  if (en) {
    f.S = (unsigned long long *)(base + off);
    off = align_up(off + cap * W * 8, 256);
  }
  if (W > 4) f.vw = (unsigned int *)(base + off);
  else f.vv = (unsigned short *)(base + off);
  f.cap = cap;
  f.cap_s = cap_s;
  return f;
}

size_t frontier_bytes(unsigned long long cap_s, int W, bool en) {
  const unsigned long long cap = cap_s * CC_SHARDS;
  size_t b = align_up(cap * W * 8, 256);
  if (en) b += align_up(cap * W * 8, 256);
  b += align_up(cap * vv_bytes(W), 256);
  return b;
}

// Carves the depth-first workspace (per-wavefront stacks, mailboxes and
// inboxes) out of a region of `bytes`.  Returns the number of wavefronts
// that fit (<= waves, a multiple of 4), 0 if not even 4 fit.
int carve_dfs(char *base, size_t bytes, int W, bool en, int waves, DfsWork *wk,
              bool batch = false) {
  DfsWork d{};
  const size_t item = (size_t)W * 8 * (en ? 3 : 2) + 4 + (batch ? 4 : 0);
  // a step pushes at most two frames per lane, after a full LDS ring (at
  // most 256 entries) has moved out below them
  const unsigned long long min_cap = 4 * CC_CHUNK + 256;
  auto need = [&](int nw, unsigned long long cap_w) {
    return (size_t)nw * (CC_MAIL * 4 + CC_CHUNK * item + cap_w * item) + 16 * 256;
  };
  int nw = waves;
  while (nw > 4 && need(nw, min_cap) > bytes) nw -= 4;
  if (need(nw, min_cap) > bytes) return 0;
  unsigned long long cap_w = (bytes - need(nw, 0)) / ((size_t)nw * item);
  cap_w = std::min<unsigned long long>(cap_w, 1ull << 20) & ~63ull;
  if (cap_w < min_cap) return 0;
  size_t off = 0;
  auto take = [&](size_t b) {
    char *q = base + off;
    off = align_up(off + b, 256);
    return q;
  };
  d.mail = (unsigned int *)take((size_t)nw * CC_MAIL * 4);
  d.inX = (unsigned long long *)take((size_t)nw * W * CC_CHUNK * 8);
  d.inE = (unsigned long long *)take((size_t)nw * W * CC_CHUNK * 8);
  if (en) d.inS = (unsigned long long *)take((size_t)nw * W * CC_CHUNK * 8);
  d.inM = (unsigned int *)take((size_t)nw * CC_CHUNK * 4);
  if (batch) d.inG = (unsigned int *)take((size_t)nw * CC_CHUNK * 4);
  d.cap_w = cap_w;
  d.stackX = (unsigned long long *)take((size_t)nw * W * cap_w * 8);
  d.stackE = (unsigned long long *)take((size_t)nw * W * cap_w * 8);
  if (en) d.stackS = (unsigned long long *)take((size_t)nw * W * cap_w * 8);
  d.stackM = (unsigned int *)take((size_t)nw * cap_w * 4);
  if (batch) d.stackG = (unsigned int *)take((size_t)nw * cap_w * 4);
  d.nwaves = nw;
  d.donate_check = 32;
  d.donate_min = 2 * CC_CHUNK;
  *wk = d;
  return nw;
}

// Depth-first diagnostics of a run from the control block's tail.
void dfs_stats(const CcCtl &h, cc_run_info *info) {
  info->dfs_steps = (int64_t)h.dfs_batches;
  info->dfs_donations = (int64_t)h.donations;
  info->dfs_lane_use = h.dfs_batches ? (double)h.dfs_lanes / (64.0 * (double)h.dfs_batches) : 0.0;
  info->dfs_idle_frac = h.dfs_wave_clk ? (double)h.dfs_idle_clk / (double)h.dfs_wave_clk : 0.0;
  info->dfs_fills = (int64_t)h.dfs_fills;
  info->dfs_spills = (int64_t)h.dfs_spills;
  info->dfs_global_adds = (int64_t)h.dfs_gatomics;
}

struct RunOut {
  OutDev out{};
  bool enumerate = false;
  // Host output: the cycles are written to device staging at the end of
  // the run's own workspace (out.verts/out.offsets are then ignored and
  // out.*_cap give the staging capacities) and copied into these host
  // buffers when they fit.
  int32_t *host_verts = nullptr;
  int64_t *host_offsets = nullptr;
  RootRange roots;  // stage-one roots the run starts from (default: all)
};

// One full device run: stage one, the level loop, and the depth-first
// continuation if the budget (or CC_FORCE_DFS) requires it.
//
// Device memory (one stream-ordered allocation): two sharded frontier
// buffers used alternately by the levels and, in enumerate mode, two staging
// buffers for the cycles one level closes and the next decodes, all sized by
// the budget; then the depth-first workspace (stacks, mailboxes, inboxes) in
// a region of its own, which no other kernel writes, zeroed before each
// depth-first pass.
cc_status run_device(cc_graph *g, const RunOut &ro) {
  const int n = g->n;
  const int W = g->W;
  const bool en = ro.enumerate;
  hipStream_t s = g->stream;
  const int64_t budget =
      g->opt.frontier_budget_bytes > 0 ? g->opt.frontier_budget_bytes : kDefaultBudget;
  // bytes per unit of capacity: a path in each frontier buffer, plus a
  // staged cycle in each of the four staging buffers
  const size_t per_unit =
      2 * ((size_t)W * 8 * (en ? 2 : 1) + vv_bytes(W)) + (en ? 4 * (size_t)W * 8 : 0);
  unsigned long long cap_s = (unsigned long long)budget / per_unit / CC_SHARDS;
  // stage one writes every initial triplet (at most sum C(deg, 2), counted
  // by the ingest) round-robin over the shards
  const unsigned long long min_cap_s =
      (unsigned long long)std::min<int64_t>(g->pairs, choose3(n)) / CC_SHARDS + CC_CHUNK;
  cap_s = align_up(std::max(cap_s, min_cap_s), 64);
  const unsigned long long cap = cap_s * CC_SHARDS;
  const size_t buf_bytes = align_up(frontier_bytes(cap_s, W, en), 1 << 16);
  const size_t stage_bytes = en ? align_up(cap * W * 8, 1 << 16) : 0;
  const size_t dfs_bytes = align_up(
      (size_t)std::min<int64_t>(std::max<int64_t>(budget / 2, (int64_t)64 << 20), (int64_t)2 << 30),
      1 << 16);
  const bool host_out = en && ro.host_offsets != nullptr;
  const size_t hv_bytes = host_out ? align_up((size_t)std::max<int64_t>(ro.out.verts_cap, 1) * 4, 256) : 0;
  const size_t ho_bytes = host_out ? align_up((size_t)(ro.out.cyc_cap + 1) * 8, 256) : 0;
  // CC_SORTED: a copy area for the vertex ids and two index arrays
  const bool sorted = en && (g->opt.flags & CC_SORTED);
  const size_t sv_bytes =
      sorted ? align_up((size_t)std::max<int64_t>(ro.out.verts_cap, 1) * 4, 256) : 0;
  const size_t si_bytes =
      sorted ? align_up((size_t)std::max<int64_t>(ro.out.cyc_cap, 1) * 4, 256) : 0;
  char *arena = nullptr;
  CC_TRY(hipMallocAsync((void **)&arena,
                        2 * buf_bytes + 4 * stage_bytes + dfs_bytes + hv_bytes + ho_bytes +
                            sv_bytes + 2 * si_bytes,
                        s));
  char *sort_region = arena + 2 * buf_bytes + 4 * stage_bytes + dfs_bytes + hv_bytes + ho_bytes;
  char *dfs_region = arena + 2 * buf_bytes + 4 * stage_bytes;
  OutDev out = ro.out;
  if (host_out) {
    out.verts = (int *)(dfs_region + dfs_bytes);
    out.offs = (long long *)(dfs_region + dfs_bytes + hv_bytes);
  }
  LevelBufs lb{};
  lb.f[0] = carve_frontier(arena, cap_s, W, en);
  lb.f[1] = carve_frontier(arena + buf_bytes, cap_s, W, en);
  Frontier *f = lb.f;
  if (en) {
    for (int i = 0; i < 4; ++i) {
      lb.st[i].C = (unsigned long long *)(arena + 2 * buf_bytes + i * stage_bytes);
      lb.st[i].cap = cap;
      lb.st[i].cap_s = cap_s;
    }
    // after a hand-over the four staging buffers are free: the depth-first
    // kernel stages its cycles there, as one array of cycle bitsets
    out.dstage = (unsigned long long *)(arena + 2 * buf_bytes);
    out.dstage_cap = (long long)(4 * stage_bytes / (8 * (size_t)W));
  }

  const int maxc = std::max(1, g->max_deg - 1);
  int waves_per_cu = g->opt.dfs_waves_per_cu > 0 ? g->opt.dfs_waves_per_cu : 24;
  waves_per_cu = std::min(std::max(waves_per_cu, 4), 32);
  // at most what is resident at once, so every wavefront of the persistent
  // grid runs from the start
  auto want_waves = [&](bool enum_pass) {
    const int wpc = std::min(waves_per_cu, 4 * cc_dfs_blocks_per_cu(W, enum_pass, false));
    return std::max(4, (g->dev.cus * wpc) / 4 * 4);
  };
  // the counting pass (wc) and, in enumerate mode, the writing pass (we)
  // use the same region one after the other
  DfsWork wc{}, we{};
  const int nw_c = carve_dfs(dfs_region, dfs_bytes, W, false, want_waves(false), &wc);
  const int nw_e = en ? carve_dfs(dfs_region, dfs_bytes, W, true, want_waves(true), &we) : 4;
  if (nw_c < 4 || nw_e < 4) {
    (void)hipFreeAsync(arena, s);
    return CC_ERR_OUT_OF_MEMORY;
  }
  for (DfsWork *d : {&wc, &we}) {
    if (g->opt.dfs_donate_min > 0) d->donate_min = g->opt.dfs_donate_min;
    d->claim = g->opt.dfs_claim > 0 ? (g->opt.dfs_claim + CC_CHUNK - 1) / CC_CHUNK * CC_CHUNK : 0;
  }
  const int dfs_blocks_c = nw_c / 4, dfs_blocks_e = nw_e / 4;
  // one resident wave of step blocks: as many per CU as registers and LDS
  // allow, at most kStepBlocksPerCu
  const int bfs_blocks =
      g->opt.bfs_blocks > 0
          ? g->opt.bfs_blocks
          : g->dev.cus * std::min(cc_step_blocks_per_cu(W, en), kStepBlocksPerCu);
  const int forced = (g->opt.flags & CC_FORCE_DFS) ? std::max(3, (int)g->opt.dfs_level) : -1;
  const unsigned long long idle_timeout =
      (unsigned long long)(kIdleTimeoutSeconds * (double)g->dev.clock_hz);

  GraphDev gd{g->d_adj, g->d_adj_orig, g->d_perm, n};
  CcCtl *ctl = g->d_ctl;
  for (double &x : g->level_ms) x = 0.0;
  hipError_t e = hipSuccess;
  int levels = 0;
  auto chk = [&](hipError_t x) {
    if (x != hipSuccess && e == hipSuccess) e = x;
  };
  const bool prof = (g->opt.flags & CC_PROFILE) != 0;
  if (prof) {
    for (int i = 0; i < 2 * n + 8; ++i)
      if (!g->evp[i]) chk(hipEventCreate(&g->evp[i]));
  }
  // evp layout: [0,1] stage one, [2+2(t-3), 3+2(t-3)] level t, [2n+2, 2n+3] depth-first
  auto mark = [&](int i) {
    if (prof) chk(hipEventRecord(g->evp[i], s));
  };
  chk(hipEventRecord(g->ev0, s));
  mark(0);
  mark(1);
  // Each step expands the paths of one length by one level, or by two when
  // its output provably fits, and (enumerate mode) decodes the cycles the
  // previous step staged.  There are at most n - 2 steps, one launch each.
  // The step kernels report the end of the loop through a pinned host word
  // and launching stops there; the host keeps at most kLevelsAhead launches
  // queued beyond the last step the device has started (waiting at most
  // kAheadWaitUs for it), so it sees the end a few steps after the frontier
  // empties.
  const bool two_ok = !(g->opt.flags & CC_ONE_LEVEL_STEPS);
  {
    volatile unsigned int *done = g->h_done;
    done[0] = 0u;
    done[1] = 0u;
    done[2] = 0u;
    done[3] = 0u;
    // Launch 0 runs stage one and the leading levels on one block with the
    // frontier in LDS; each later launch runs one step, so n - 2 of them
    // are enough.
    mark(2);
    const size_t head_lds = head_dyn_lds(W, en, g->dev.lds_block);
    chk(cc_launch_head(W, en, gd, ctl, lb, out, forced, head_lds, g->d_done, true, ro.roots, s));
    mark(3);
    ++levels;
    for (int launch = 1; launch < n - 1 && e == hipSuccess; ++launch, ++levels) {
      if (launch >= kLevelsAhead) {
        const auto t_wait = std::chrono::steady_clock::now();
        while (done[0] == 0u && (int)done[1] < launch - kLevelsAhead + 1 &&
               std::chrono::steady_clock::now() - t_wait <
                   std::chrono::microseconds(kAheadWaitUs)) {
        }
      }
      if (done[0] != 0u) break;
      mark(2 + 2 * launch);
      chk(cc_launch_step(W, en, gd, ctl, lb, out, launch, forced, maxc, two_ok, bfs_blocks,
                         g->d_done, s));
      mark(3 + 2 * launch);
    }
  }
  // Depth-first continuation.  Each of its kernels returns at once if the
  // levels finished within the budget; they are not launched at all when
  // the host has already seen the loop end without a hand-over (the
  // hand-over word is released before the end-of-loop word).
  volatile unsigned int *hd = g->h_done;
  const bool levels_finished = hd[0] != 0u && hd[2] == 0u;
  mark(2 * n + 2);
  if (levels_finished) {
    // nothing to continue
  } else if (!en) {
    chk(cc_launch_dfs_prepare(ctl, wc, n, false, s));
    chk(cc_launch_dfs(W, false, gd, ctl, f[0], f[1], wc, out,
                      dev_field(ctl, offsetof(CcCtl, hist_sh)), CC_HSLOTS, true, dfs_blocks_c,
                      idle_timeout, s));
  } else {
    chk(cc_launch_dfs_prepare(ctl, wc, n, false, s));
    chk(cc_launch_dfs(W, false, gd, ctl, f[0], f[1], wc, out,
                      dev_field(ctl, offsetof(CcCtl, dfs_hist)), 0, true, dfs_blocks_c,
                      idle_timeout, s));
    chk(cc_launch_dfs_prepare(ctl, we, n, true, s));
    chk(cc_launch_dfs(W, true, gd, ctl, f[0], f[1], we, out, nullptr, 0, false,
                      dfs_blocks_e, idle_timeout, s));
    chk(cc_launch_dfs_decode(W, gd, ctl, out, g->dev.cus * 4, s));
  }
  mark(2 * n + 3);
  // the step that found the frontier empty has already finalized when it
  // says so (host_done[3], released before the end-of-loop word)
  if (!(levels_finished && hd[3] != 0u)) chk(cc_launch_finalize(ctl, out, n, en, s));
  if (sorted)
    chk(cc_launch_sort_cycles(ctl, out, n, (int *)sort_region, (unsigned *)(sort_region + sv_bytes),
                              (unsigned *)(sort_region + sv_bytes + si_bytes), s));
  chk(hipEventRecord(g->ev1, s));
  // Read back the unsharded tail of the control block (everything for
  // profiling runs, which also report per-level traffic).
  const size_t tail = prof ? 0 : offsetof(CcCtl, hist);
  chk(hipMemcpyAsync((char *)g->h_ctl + tail, (char *)ctl + tail, sizeof(CcCtl) - tail,
                     hipMemcpyDeviceToHost, s));
  if (!host_out) chk(hipFreeAsync(arena, s));
  chk(hipStreamSynchronize(s));
  if (e != hipSuccess) {
    if (host_out) (void)hipFreeAsync(arena, s);
    return hip_err(e);
  }

  const CcCtl &h = *g->h_ctl;
  std::memset(g->hist, 0, sizeof(g->hist));
  std::memset(g->front, 0, sizeof(g->front));
  int64_t cycles = 0, paths = 0;
  for (int k = 0; k <= n; ++k) {
    g->hist[k] = (int64_t)h.hist[k];
    g->front[k] = (int64_t)h.front[k];
    cycles += g->hist[k];
    paths += g->front[k];
  }
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, g->ev0, g->ev1);
  g->info.cycles = cycles;
  g->info.paths = paths;
  g->info.peak_frontier = (int64_t)h.peak;
  g->info.switch_level = h.mode ? h.switch_level : 0;
  // launch 0 of the launched loop is the one-block head kernel
  g->info.levels_launched = std::max(levels - 1, 0);
  const int launches = levels;
  const int head_steps = std::max(h.head_steps, 0);
  levels = std::min(std::max(h.levels_run, 0), CC_HSLOTS - 1);  // steps run
  g->info.head_steps = head_steps;
  g->info.gpu_ms = ms;
  g->info.stage1_ms = g->info.level_ms = g->info.dfs_ms = g->info.head_ms = 0.0;
  g->info.level_bytes = g->info.head_bytes = 0;
  if (prof) {
    auto span = [&](int a, int b) {
      float x = 0.f;
      (void)hipEventElapsedTime(&x, g->evp[a], g->evp[b]);
      return (double)x;
    };
    g->info.stage1_ms = span(0, 1);
    // per-step device time, credited to the length t the step expanded
    // (CcCtl::step_level); a two-level step's time goes to its t, and a
    // launch that ran several small steps is credited to its first
    const int steps = levels;
    auto step_t = [&](int st) { return st < CC_HSLOTS ? h.step_level[st] : 0; };
    for (int li = 0; li < launches; ++li) {
      const double ms_s = span(2 + 2 * li, 3 + 2 * li);
      (li == 0 ? g->info.head_ms : g->info.level_ms) += ms_s;
      const int first = li == 0 ? 0 : (li < CC_HSLOTS ? h.launch_step[li] - 1 : -1);
      const int t = first >= 0 ? step_t(first) : 0;
      if (t >= 3 && t < CC_HSLOTS) g->level_ms[t] += ms_s;
    }
    g->info.dfs_ms = span(2 * n + 2, 2 * n + 3);
    // Bytes the steps must move: each path a step expands is read once and
    // each path it writes is written once (X words, S words in enumerate
    // mode, 2 bytes of end vertices); each cycle is staged (W words written,
    // then read by the next step) and written as k int32 ids plus one int64
    // offset.  Paths a two-level step only counts move no bytes.
    const int64_t pp = (int64_t)W * 8 * (en ? 2 : 1) + 2;
    auto level_count = [&](int t) {
      unsigned long long c = 0;
      for (int sh = 0; sh < CC_SHARDS; ++sh) c += std::min(h.count_sh[sh][t], cap_s);
      return (int64_t)c;
    };
    const int last_len = h.mode ? h.bfs_max_len : n;
    for (int st = 0; st < steps; ++st) {
      const int t = step_t(st);
      if (t < 3 || t > n) continue;
      const int tn = (st + 1 < steps && st + 1 < CC_HSLOTS) ? step_t(st + 1) : t + 1;
      if (tn <= t) continue;
      int64_t bytes = level_count(t) * pp;
      if (tn <= n && st + 1 < steps) bytes += level_count(tn) * pp;
      if (en)
        for (int k = t + 1; k <= tn && k <= n && k <= last_len; ++k)
          bytes += (int64_t)h.hist[k] * (16 * W + 4 * k + 8);
      (st < head_steps ? g->info.head_bytes : g->info.level_bytes) += bytes;
    }
  }
  g->have_run = true;
  g->info.device_diag = (int64_t)h.diag;
  dfs_stats(h, &g->info);
  cc_status st = CC_OK;
  if (h.status & (CC_DEV_CORRUPT | CC_DEV_LOST))
    st = CC_ERR_INTERNAL;
  else if (h.status & CC_DEV_STACK_FULL)
    st = CC_ERR_OUT_OF_MEMORY;
  // the whole graph's histogram, unless the run started from part of its roots
  g->hist_ok = st == CC_OK && ro.roots.lo == 0 && ro.roots.hi == RootRange{}.hi;
  if (host_out) {
    // what the run wrote: the cycles of the output window
    int64_t cw = 0, vw = 0;
    for (int k = 0; k <= n; ++k)
      if (k >= out.kmin && k <= out.kmax) {
        cw += g->hist[k];
        vw += g->hist[k] * k;
      }
    if (st == CC_OK && cw <= out.cyc_cap && vw <= out.verts_cap) {
      if (hipMemcpyAsync(ro.host_verts, out.verts, (size_t)vw * 4, hipMemcpyDeviceToHost, s) !=
              hipSuccess ||
          hipMemcpyAsync(ro.host_offsets, out.offs, (size_t)(cw + 1) * 8,
                         hipMemcpyDeviceToHost, s) != hipSuccess)
        st = CC_ERR_DEVICE;
    }
    if (hipFreeAsync(arena, s) != hipSuccess && st == CC_OK) st = CC_ERR_DEVICE;
    if (hipStreamSynchronize(s) != hipSuccess && st == CC_OK) st = CC_ERR_DEVICE;
  }
  return st;
}

cc_status check_handle(cc_graph *g) {
  if (!g) return CC_ERR_INVALID_ARG;
  if (hipSetDevice(g->device) != hipSuccess) return CC_ERR_DEVICE;
  return CC_OK;
}

cc_status run_counts(cc_graph *g, RootRange roots = RootRange{}) {
  if (g->n < 3) {
    std::memset(g->hist, 0, sizeof(g->hist));
    std::memset(g->front, 0, sizeof(g->front));
    g->info = cc_run_info{};
    g->have_run = true;
    return CC_OK;
  }
  RunOut ro;
  ro.roots = roots;
  return run_device(g, ro);
}

}  // namespace

extern "C" {

int32_t cc_abi_version(void) { return CC_ABI_VERSION; }

const char *cc_status_string(cc_status s) {
  switch (s) {
    case CC_OK: return "ok";
    case CC_ERR_INVALID_ARG: return "invalid argument";
    case CC_ERR_NOT_SIMPLE: return "graph is not a simple undirected graph";
    case CC_ERR_TOO_LARGE: return "graph has more vertices than supported";
    case CC_ERR_BUFFER_TOO_SMALL: return "output buffer too small";
    case CC_ERR_OUT_OF_MEMORY: return "out of device memory or frontier budget too small";
    case CC_ERR_DEVICE: return "HIP runtime or device error";
    case CC_ERR_NO_DEVICE: return "no usable gfx950 device";
    case CC_ERR_NOT_READY: return "request not finished yet";
    case CC_ERR_INTERNAL: return "device-side consistency check failed; results discarded";
  }
  return "unknown status";
}

cc_status cc_prepare(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                     const cc_options *opt, cc_graph **out) {
  if (!out) return CC_ERR_INVALID_ARG;
  *out = nullptr;
  if (n < 0) return CC_ERR_INVALID_ARG;
  if (n > CC_MAX_VERTICES) return CC_ERR_TOO_LARGE;
  if (n > 0 && !row_ptr) return CC_ERR_INVALID_ARG;
  const uint32_t flags = opt ? opt->flags : 0u;
  if (flags & ~(CC_INPUT_DEVICE | CC_OUTPUT_DEVICE | CC_FORCE_DFS | CC_PROFILE | CC_ONE_LEVEL_STEPS |
                CC_SORTED))
    return CC_ERR_INVALID_ARG;
  if (opt && (opt->frontier_budget_bytes < 0 || opt->dfs_donate_min < 0 || opt->dfs_claim < 0 ||
              opt->dfs_waves_per_cu < 0 || opt->bfs_blocks < 0))
    return CC_ERR_INVALID_ARG;
  if ((flags & CC_FORCE_DFS) && opt->dfs_level < 3) return CC_ERR_INVALID_ARG;
  int64_t nnz = 0;
  if (n > 0 && !(flags & CC_INPUT_DEVICE)) {
    nnz = row_ptr[n];
    if (row_ptr[0] != 0 || nnz < 0 || nnz > (int64_t)n * (n - 1)) return CC_ERR_NOT_SIMPLE;
    if (nnz > 0 && !col_idx) return CC_ERR_INVALID_ARG;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return CC_ERR_NO_DEVICE;
  DeviceInfo di;
  cc_status st = device_info(dev, &di);
  if (st != CC_OK) return st;

  cc_graph *g = new cc_graph();
  g->device = dev;
  g->dev = di;
  if (opt) g->opt = *opt;
  g->stream = (hipStream_t)g->opt.stream;
  g->n = n;
  g->W = words_for(n);
  const size_t adj_b = align_up((size_t)CC_MAXN * CC_MAXN / 8, 256);  // n rows of W words
  const size_t vec_b = align_up((size_t)CC_MAXN * 4, 256);
  const size_t ctl_b = align_up(sizeof(CcCtl), 256);
  // staging for a host CSR (at most CC_MAXN rows and CC_MAXN (CC_MAXN - 1)
  // entries), so preparing a handle allocates nothing after warm-up and
  // never splits the stream-ordered pool that holds the run arenas
  const size_t rp_b = align_up((size_t)(CC_MAXN + 1) * 4, 256);
  const size_t ci_b = align_up((size_t)CC_MAXN * (CC_MAXN - 1) * 4, 256);
  const size_t blob = 2 * adj_b + 2 * vec_b + 256 + ctl_b + rp_b + ci_b;
  auto fail = [&](cc_status s) {
    cc_release(g);
    return s;
  };
  HandleRes res;
  if (pool_take(dev, &res)) {
    g->d_blob = res.d_blob;
    g->h_ctl = (CcCtl *)res.h_ctl;
    g->h_done = (unsigned int *)res.h_done;
    g->ev0 = res.ev0;
    g->ev1 = res.ev1;
  } else {
    if (hipMalloc(&g->d_blob, blob) != hipSuccess) return fail(CC_ERR_OUT_OF_MEMORY);
    if (hipHostMalloc((void **)&g->h_ctl, sizeof(CcCtl), hipHostMallocDefault) != hipSuccess)
      return fail(CC_ERR_OUT_OF_MEMORY);
    if (hipHostMalloc((void **)&g->h_done, 64, hipHostMallocMapped | hipHostMallocCoherent) !=
        hipSuccess)
      return fail(CC_ERR_OUT_OF_MEMORY);
    if (hipEventCreate(&g->ev0) != hipSuccess || hipEventCreate(&g->ev1) != hipSuccess)
      return fail(CC_ERR_DEVICE);
  }
  if (hipHostGetDevicePointer((void **)&g->d_done, g->h_done, 0) != hipSuccess)
    return fail(CC_ERR_DEVICE);
  char *b = (char *)g->d_blob;
  g->d_adj = (unsigned long long *)b;
  g->d_adj_orig = (unsigned long long *)(b + adj_b);
  g->d_perm = (int *)(b + 2 * adj_b);
  g->d_label = (int *)(b + 2 * adj_b + vec_b);
  g->d_status = (unsigned int *)(b + 2 * adj_b + 2 * vec_b);
  g->d_ctl = (CcCtl *)(b + 2 * adj_b + 2 * vec_b + 256);
  if (n == 0) {
    *out = g;
    return CC_OK;
  }
  const int *d_rp = row_ptr, *d_ci = col_idx;
  hipStream_t s = g->stream;
  if (!(flags & CC_INPUT_DEVICE)) {
    // nnz <= n (n - 1) was checked above, so the CSR fits the staging area
    int *st_rp = (int *)(b + 2 * adj_b + 2 * vec_b + 256 + ctl_b);
    int *st_ci = (int *)((char *)st_rp + rp_b);
    if (hipMemcpyAsync(st_rp, row_ptr, (size_t)(n + 1) * 4, hipMemcpyHostToDevice, s) != hipSuccess ||
        (nnz > 0 && hipMemcpyAsync(st_ci, col_idx, (size_t)nnz * 4, hipMemcpyHostToDevice, s) !=
                        hipSuccess)) {
      (void)hipStreamSynchronize(s);
      return fail(CC_ERR_DEVICE);
    }
    d_rp = st_rp;
    d_ci = st_ci;
  }
  // status word, then (8 bytes on) the sum over vertices of C(deg, 2),
  // which bounds the initial triplets and triangles
  long long *d_pairs = (long long *)((char *)g->d_status + 8);
  // The ingest also answers in mapped host memory (words kReplyWord.. of
  // the pinned flag area), which the host polls: cheaper than a copy and a
  // stream synchronisation.  The stream may hold earlier work of the
  // caller's, so polling gives way to a synchronisation after kReplySpinUs.
  volatile unsigned int *rep = g->h_done + kReplyWord;
  rep[0] = 0u;
  std::atomic_thread_fence(std::memory_order_seq_cst);
  hipError_t e = cc_launch_ingest(g->W, 1, nullptr, n, d_rp, d_ci, g->d_adj, g->d_adj_orig, g->d_perm,
                                  g->d_label, g->d_status, d_pairs, g->d_done + kReplyWord, s);
  if (e == hipSuccess) {
    const auto t0 = std::chrono::steady_clock::now();
    while (rep[0] == 0u &&
           std::chrono::steady_clock::now() - t0 < std::chrono::microseconds(kReplySpinUs)) {
    }
    if (rep[0] == 0u) e = hipStreamSynchronize(s);
  }
  if (e != hipSuccess) return fail(hip_err(e));
  if (rep[0] == 0u) return fail(CC_ERR_DEVICE);
  std::atomic_thread_fence(std::memory_order_acquire);
  const unsigned int stv = rep[1];
  if ((stv & 0xffu) != 0u || !(stv & 0x100u)) return fail(CC_ERR_NOT_SIMPLE);
  g->max_deg = (int)(stv >> 16);
  g->pairs = (int64_t)((unsigned long long)rep[2] | ((unsigned long long)rep[3] << 32));
  *out = g;
  return CC_OK;
}

cc_status cc_histogram(cc_graph *g, int64_t *hist, int32_t hist_len) {
  cc_status st = check_handle(g);
  if (st != CC_OK) return st;
  if (!hist || hist_len < g->n + 1) return CC_ERR_INVALID_ARG;
  st = run_counts(g);
  if (st != CC_OK) return st;
  for (int k = 0; k < hist_len; ++k) hist[k] = k <= g->n ? g->hist[k] : 0;
  return CC_OK;
}

cc_status cc_count(cc_graph *g, int64_t *total) {
  cc_status st = check_handle(g);
  if (st != CC_OK) return st;
  if (!total) return CC_ERR_INVALID_ARG;
  st = run_counts(g);
  if (st != CC_OK) return st;
  *total = g->info.cycles;
  return CC_OK;
}

cc_status cc_enumerate(cc_graph *g, int32_t *verts, int64_t verts_cap, int64_t *offsets,
                       int64_t cycles_cap, int64_t *n_cycles, int64_t *n_verts) {
  cc_status st = check_handle(g);
  if (st != CC_OK) return st;
  if (!n_cycles || !n_verts || verts_cap < 0 || cycles_cap < 0) return CC_ERR_INVALID_ARG;
  if ((verts_cap > 0 && !verts) || !offsets) return CC_ERR_INVALID_ARG;
  *n_cycles = 0;
  *n_verts = 0;
  const bool dev_out = (g->opt.flags & CC_OUTPUT_DEVICE) != 0;
  if (g->n < 3) {
    (void)run_counts(g);
    if (dev_out) {
      const int64_t zero = 0;
      if (hipMemcpyAsync(offsets, &zero, 8, hipMemcpyHostToDevice, g->stream) != hipSuccess ||
          hipStreamSynchronize(g->stream) != hipSuccess)
        return CC_ERR_DEVICE;
    } else {
      offsets[0] = 0;
    }
    return CC_OK;
  }
  auto totals = [&](int64_t *c, int64_t *v) {
    *c = 0;
    *v = 0;
    for (int k = 0; k <= g->n; ++k) {
      *c += g->hist[k];
      *v += g->hist[k] * k;
    }
  };
  if (dev_out) {
    RunOut ro;
    ro.enumerate = true;
    ro.out = OutDev{verts, (long long *)offsets, verts_cap, cycles_cap};
    st = run_device(g, ro);
    if (st != CC_OK) return st;
    totals(n_cycles, n_verts);
    if (*n_cycles > cycles_cap || *n_verts > verts_cap) return CC_ERR_BUFFER_TOO_SMALL;
    return CC_OK;
  }
  // Host buffers: the run writes into device staging of the caller's
  // capacities, carved from its own workspace, and copies back what it
  // wrote.  Capacities beyond kHostStageBytes are sized exactly by a
  // counting run first.
  RunOut ro;
  ro.enumerate = true;
  ro.host_verts = verts;
  ro.host_offsets = offsets;
  const double want = (double)verts_cap * 4 + ((double)cycles_cap + 1) * 8;
  if (want <= (double)kHostStageBytes) {
    ro.out = OutDev{nullptr, nullptr, verts_cap, cycles_cap};
  } else {
    st = run_counts(g);
    if (st != CC_OK) return st;
    int64_t c = 0, v = 0;
    totals(&c, &v);
    if (c > cycles_cap || v > verts_cap) {
      *n_cycles = c;
      *n_verts = v;
      return CC_ERR_BUFFER_TOO_SMALL;
    }
    ro.out = OutDev{nullptr, nullptr, v, c};
  }
  st = run_device(g, ro);
  if (st != CC_OK) return st;
  totals(n_cycles, n_verts);
  if (*n_cycles > cycles_cap || *n_verts > verts_cap) return CC_ERR_BUFFER_TOO_SMALL;
  return CC_OK;
}

cc_status cc_enumerate_lengths(cc_graph *g, int32_t k_min, int32_t k_max, int32_t *verts,
                               int64_t verts_cap, int64_t *offsets, int64_t cycles_cap,
                               int64_t *n_cycles, int64_t *n_verts) {
  cc_status st = check_handle(g);
  if (st != CC_OK) return st;
  if (!n_cycles || !n_verts || verts_cap < 0 || cycles_cap < 0 || k_min < 0 || k_max < k_min)
    return CC_ERR_INVALID_ARG;
  if ((verts_cap > 0 && !verts) || !offsets) return CC_ERR_INVALID_ARG;
  *n_cycles = 0;
  *n_verts = 0;
  const bool dev_out = (g->opt.flags & CC_OUTPUT_DEVICE) != 0;
  if (g->n >= 3 && !g->hist_ok) {
    // sizes of the window: the histogram, from a counting run if no
    // complete run has produced it yet
    st = run_counts(g);
    if (st != CC_OK) return st;
  }
  int64_t cshift = 0, vshift = 0, cw = 0, vw = 0;
  if (g->n >= 3)
    for (int k = 0; k <= g->n; ++k) {
      if (k < k_min) {
        cshift += g->hist[k];
        vshift += g->hist[k] * k;
      } else if (k <= k_max) {
        cw += g->hist[k];
        vw += g->hist[k] * k;
      }
    }
  *n_cycles = cw;
  *n_verts = vw;
  if (cw > cycles_cap || vw > verts_cap) return CC_ERR_BUFFER_TOO_SMALL;
  if (cw == 0) {
    // nothing in the window: only the closing offset
    if (dev_out) {
      const int64_t zero = 0;
      if (hipMemcpyAsync(offsets, &zero, 8, hipMemcpyHostToDevice, g->stream) != hipSuccess ||
          hipStreamSynchronize(g->stream) != hipSuccess)
        return CC_ERR_DEVICE;
    } else {
      offsets[0] = 0;
    }
    return CC_OK;
  }
  RunOut ro;
  ro.enumerate = true;
  if (dev_out) {
    ro.out = OutDev{verts, (long long *)offsets, verts_cap, cycles_cap};
  } else {
    ro.host_verts = verts;
    ro.host_offsets = offsets;
    ro.out = OutDev{nullptr, nullptr, vw, cw};
  }
  ro.out.kmin = k_min;
  ro.out.kmax = k_max;
  ro.out.cshift = cshift;
  ro.out.vshift = vshift;
  return run_device(g, ro);
}

cc_status cc_root_total(cc_graph *g, int64_t *n_roots) {
  cc_status st = check_handle(g);
  if (st != CC_OK) return st;
  if (!n_roots) return CC_ERR_INVALID_ARG;
  *n_roots = 0;
  if (g->n < 3) return CC_OK;
  if (g->n_roots >= 0) {
    *n_roots = g->n_roots;
    return CC_OK;
  }
  // computed into the handle's status area (after the status word and the
  // pair bound), then read back
  long long *d_out = (long long *)((char *)g->d_status + 16);
  long long v = 0;
  GraphDev gd{g->d_adj, g->d_adj_orig, g->d_perm, g->n};
  if (cc_launch_root_total(g->W, gd, d_out, g->stream) != hipSuccess ||
      hipMemcpyAsync(&v, d_out, 8, hipMemcpyDeviceToHost, g->stream) != hipSuccess ||
      hipStreamSynchronize(g->stream) != hipSuccess)
    return CC_ERR_DEVICE;
  *n_roots = v;
  g->n_roots = v;
  return CC_OK;
}

cc_status cc_histogram_roots(cc_graph *g, int64_t root_lo, int64_t root_hi, int64_t *hist,
                             int32_t hist_len) {
  cc_status st = check_handle(g);
  if (st != CC_OK) return st;
  if (!hist || hist_len < g->n + 1 || root_lo < 0 || root_hi < root_lo)
    return CC_ERR_INVALID_ARG;
  st = run_counts(g, RootRange{root_lo, root_hi});
  if (st != CC_OK) return st;
  for (int k = 0; k < hist_len; ++k) hist[k] = k <= g->n ? g->hist[k] : 0;
  return CC_OK;
}

cc_status cc_enumerate_by_roots(cc_graph *g, int32_t *verts, int64_t verts_cap, int64_t *offsets,
                                int64_t cycles_cap, int64_t *root_first, int64_t roots_cap,
                                int64_t *n_cycles, int64_t *n_verts) {
  cc_status st = check_handle(g);
  if (st != CC_OK) return st;
  if (!n_cycles || !n_verts || verts_cap < 0 || cycles_cap < 0 || roots_cap < 1)
    return CC_ERR_INVALID_ARG;
  if ((verts_cap > 0 && !verts) || !offsets || !root_first) return CC_ERR_INVALID_ARG;
  *n_cycles = 0;
  *n_verts = 0;
  const bool dev_out = (g->opt.flags & CC_OUTPUT_DEVICE) != 0;
  int64_t R = 0;
  st = cc_root_total(g, &R);
  if (st != CC_OK) return st;
  if (roots_cap < R + 1) return CC_ERR_INVALID_ARG;
  hipStream_t s = g->stream;
  if (g->n < 3 || R == 0) {
    if (g->n < 3) (void)run_counts(g);
    const int64_t zero = 0;
    if (dev_out) {
      if (hipMemcpyAsync(offsets, &zero, 8, hipMemcpyHostToDevice, s) != hipSuccess ||
          hipMemcpyAsync(root_first, &zero, 8, hipMemcpyHostToDevice, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess)
        return CC_ERR_DEVICE;
    } else {
      offsets[0] = 0;
      root_first[0] = 0;
    }
    return CC_OK;
  }
  // the enumeration, ordered by length as cc_enumerate writes it, into
  // device staging of the caller's capacities
  const size_t tv_b = align_up((size_t)std::max<int64_t>(verts_cap, 1) * 4, 256);
  const size_t to_b = align_up((size_t)(cycles_cap + 1) * 8, 256);
  char *stage = nullptr;
  if (hipMallocAsync((void **)&stage, tv_b + to_b, s) != hipSuccess) return CC_ERR_OUT_OF_MEMORY;
  RunOut ro;
  ro.enumerate = true;
  ro.out = OutDev{(int *)stage, (long long *)(stage + tv_b), verts_cap, cycles_cap};
  st = run_device(g, ro);
  int64_t nc = 0, nv = 0;
  for (int k = 0; k <= g->n; ++k) {
    nc += g->hist[k];
    nv += g->hist[k] * k;
  }
  if (st == CC_OK && (nc > cycles_cap || nv > verts_cap)) {
    *n_cycles = nc;
    *n_verts = nv;
    st = CC_ERR_BUFFER_TOO_SMALL;
  }
  if (st != CC_OK) {
    (void)hipFreeAsync(stage, s);
    (void)hipStreamSynchronize(s);
    return st;
  }
  // regrouped into the caller's buffers (through device buffers of the
  // exact sizes for host output)
  const size_t work_b = align_up(cc_group_roots_workspace(nc), 256);
  const size_t vn_b = align_up((size_t)std::max<int64_t>(nv, 1) * 4, 256);
  const size_t on_b = align_up((size_t)(nc + 1) * 8, 256);
  const size_t fn_b = align_up((size_t)(R + 1) * 8, 256);
  char *work = nullptr;
  if (hipMallocAsync((void **)&work, work_b + (dev_out ? 0 : vn_b + on_b + fn_b), s) != hipSuccess) {
    (void)hipFreeAsync(stage, s);
    (void)hipStreamSynchronize(s);
    return CC_ERR_OUT_OF_MEMORY;
  }
  int *vn = dev_out ? verts : (int *)(work + work_b);
  long long *on = dev_out ? (long long *)offsets : (long long *)(work + work_b + vn_b);
  long long *fn = dev_out ? (long long *)root_first : (long long *)(work + work_b + vn_b + on_b);
  GraphDev gd{g->d_adj, g->d_adj_orig, g->d_perm, g->n};
  hipError_t e = cc_launch_group_roots(g->W, gd, g->d_label, (const int *)stage,
                                       (const long long *)(stage + tv_b), nc, R, vn, on, fn, work,
                                       s);
  long long *h_last = (long long *)(g->h_done + kGroupWord);
  *h_last = -1;
  if (e == hipSuccess && !dev_out) {
    e = hipMemcpyAsync(verts, vn, (size_t)nv * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(offsets, on, (size_t)(nc + 1) * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(root_first, fn, (size_t)(R + 1) * 8, hipMemcpyDeviceToHost, s);
  }
  if (e == hipSuccess) e = hipMemcpyAsync(h_last, fn + R, 8, hipMemcpyDeviceToHost, s);
  (void)hipFreeAsync(work, s);
  (void)hipFreeAsync(stage, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  else (void)hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_err(e);
  // every cycle got a root (first[R] == nc)
  if (*h_last != nc) return CC_ERR_INTERNAL;
  *n_cycles = nc;
  *n_verts = nv;
  return CC_OK;
}

cc_status cc_enumerate_roots(cc_graph *g, int64_t root_lo, int64_t root_hi, int32_t *verts,
                             int64_t verts_cap, int64_t *offsets, int64_t cycles_cap,
                             int64_t *n_cycles, int64_t *n_verts) {
  cc_status st = check_handle(g);
  if (st != CC_OK) return st;
  if (!n_cycles || !n_verts || verts_cap < 0 || cycles_cap < 0 || root_lo < 0 ||
      root_hi < root_lo)
    return CC_ERR_INVALID_ARG;
  if ((verts_cap > 0 && !verts) || !offsets) return CC_ERR_INVALID_ARG;
  *n_cycles = 0;
  *n_verts = 0;
  const bool dev_out = (g->opt.flags & CC_OUTPUT_DEVICE) != 0;
  const RootRange rr{root_lo, root_hi};
  auto totals = [&](int64_t *c, int64_t *v) {
    *c = 0;
    *v = 0;
    for (int k = 0; k <= g->n; ++k) {
      *c += g->hist[k];
      *v += g->hist[k] * k;
    }
  };
  if (g->n < 3 || root_lo == root_hi) {
    if (g->n < 3) (void)run_counts(g);
    if (dev_out) {
      const int64_t zero = 0;
      if (hipMemcpyAsync(offsets, &zero, 8, hipMemcpyHostToDevice, g->stream) != hipSuccess ||
          hipStreamSynchronize(g->stream) != hipSuccess)
        return CC_ERR_DEVICE;
    } else {
      offsets[0] = 0;
    }
    return CC_OK;
  }
  RunOut ro;
  ro.enumerate = true;
  ro.roots = rr;
  if (dev_out) {
    ro.out = OutDev{verts, (long long *)offsets, verts_cap, cycles_cap};
  } else {
    // host buffers: the range's exact sizes first (a counting run of the
    // same roots), then the run writes device staging of those sizes
    st = run_counts(g, rr);
    if (st != CC_OK) return st;
    int64_t c = 0, v = 0;
    totals(&c, &v);
    if (c > cycles_cap || v > verts_cap) {
      *n_cycles = c;
      *n_verts = v;
      return CC_ERR_BUFFER_TOO_SMALL;
    }
    ro.host_verts = verts;
    ro.host_offsets = offsets;
    ro.out = OutDev{nullptr, nullptr, v, c};
  }
  st = run_device(g, ro);
  if (st != CC_OK) return st;
  totals(n_cycles, n_verts);
  if (*n_cycles > cycles_cap || *n_verts > verts_cap) return CC_ERR_BUFFER_TOO_SMALL;
  return CC_OK;
}

cc_status cc_labels(cc_graph *g, int32_t *labels) {
  cc_status st = check_handle(g);
  if (st != CC_OK) return st;
  if (!labels) return CC_ERR_INVALID_ARG;
  if (g->n == 0) return CC_OK;
  if (hipMemcpyAsync(labels, g->d_label, (size_t)g->n * 4, hipMemcpyDeviceToHost, g->stream) !=
          hipSuccess ||
      hipStreamSynchronize(g->stream) != hipSuccess)
    return CC_ERR_DEVICE;
  return CC_OK;
}

cc_status cc_frontier(cc_graph *g, int64_t *front, int32_t len) {
  if (!g || !front || len < g->n + 1) return CC_ERR_INVALID_ARG;
  for (int t = 0; t < len; ++t) front[t] = (t <= g->n && g->have_run) ? g->front[t] : 0;
  return CC_OK;
}

cc_status cc_last_run(cc_graph *g, cc_run_info *info) {
  if (!g || !info) return CC_ERR_INVALID_ARG;
  *info = g->info;
  return CC_OK;
}

cc_status cc_level_times(cc_graph *g, double *ms, int32_t len) {
  if (!g || !ms || len < g->n + 1) return CC_ERR_INVALID_ARG;
  for (int t = 0; t < len; ++t) ms[t] = (t < CC_HSLOTS && g->have_run) ? g->level_ms[t] : 0.0;
  return CC_OK;
}

void cc_release(cc_graph *g) {
  if (!g) return;
  (void)hipSetDevice(g->device);
  if (g->d_blob) (void)hipStreamSynchronize(g->stream);
  for (hipEvent_t &ev : g->evp)
    if (ev) (void)hipEventDestroy(ev);
  const bool complete = g->d_blob && g->h_ctl && g->h_done && g->ev0 && g->ev1;
  if (!(complete &&
        pool_give(HandleRes{g->device, g->d_blob, g->h_ctl, g->h_done, g->ev0, g->ev1}))) {
    if (g->d_blob) (void)hipFree(g->d_blob);
    if (g->h_ctl) (void)hipHostFree(g->h_ctl);
    if (g->h_done) (void)hipHostFree(g->h_done);
    if (g->ev0) (void)hipEventDestroy(g->ev0);
    if (g->ev1) (void)hipEventDestroy(g->ev1);
  }
  delete g;
}

}  // extern "C"

// ------------------------------------------------------------------ batches
struct cc_batch {
  int device = 0;
  hipStream_t stream = nullptr;
  cc_options opt{};
  DeviceInfo dev{};
  int32_t G = 0;
  int32_t N = 0;
  int W = 1;
  int max_n = 0;
  int max_deg = 0;
  std::vector<int32_t> vtx_off;        // host copy
  std::vector<long long> root_off;     // host copy, [G+1]
  BatchRes res;                        // recycled device blob, pinned staging, events
  void *d_blob = nullptr;              // vtx_off | root_off | adj | adj_orig | perm | label | status | bound | ctl
  // pinned staging (in res.h_stage) for the host copies of a pass
  int32_t *s_off = nullptr;            // [G+1] vertex offsets
  int32_t *s_nnz = nullptr;            // adjacency entries of a device CSR
  unsigned int *s_stat = nullptr;      // [G] ingest status words
  long long *s_bound = nullptr;        // [G] sum over vertices of C(deg, 2)
  long long *s_root = nullptr;         // [G+1] root slot offsets
  unsigned long long *s_hist = nullptr;  // [G * (max_n + 2)] histograms
  int *d_vtx_off = nullptr;
  long long *d_root_off = nullptr;
  unsigned long long *d_adj = nullptr;
  unsigned long long *d_adj_orig = nullptr;
  int *d_perm = nullptr;
  int *d_label = nullptr;
  unsigned int *d_status = nullptr;
  long long *d_bound = nullptr;
  CcCtl *d_ctl = nullptr;
  CcCtl *h_ctl = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  hipEvent_t evp[4] = {};  // CC_PROFILE: around stage one and the depth-first kernel
  cc_run_info info{};
};

extern "C" {

void cc_release_batch(cc_batch *b) {
  if (!b) return;
  (void)hipSetDevice(b->device);
  // the stream's work on the blob and staging ends before they are reused
  if (b->res.device >= 0) (void)hipStreamSynchronize(b->stream);
  batch_res_give(b->res);
  delete b;
}

cc_status cc_prepare_batch(int32_t n_graphs, const int32_t *graph_vtx_off, const int32_t *row_ptr,
                           const int32_t *col_idx, const cc_options *opt, cc_batch **out) {
  if (!out) return CC_ERR_INVALID_ARG;
  *out = nullptr;
  if (n_graphs < 0 || !graph_vtx_off || (n_graphs > 0 && !row_ptr)) return CC_ERR_INVALID_ARG;
  const uint32_t flags = opt ? opt->flags : 0u;
  if (flags & ~(CC_INPUT_DEVICE | CC_OUTPUT_DEVICE | CC_PROFILE))
    return CC_ERR_INVALID_ARG;
  if (opt && (opt->frontier_budget_bytes < 0 || opt->dfs_donate_min < 0 || opt->dfs_claim < 0 ||
              opt->dfs_waves_per_cu < 0 || opt->bfs_blocks < 0))
    return CC_ERR_INVALID_ARG;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return CC_ERR_NO_DEVICE;
  DeviceInfo di;
  cc_status st = device_info(dev, &di);
  if (st != CC_OK) return st;
  cc_batch *b = new cc_batch();
  auto fail = [&](cc_status s2) {
    cc_release_batch(b);
    return s2;
  };
  b->device = dev;
  b->dev = di;
  if (opt) b->opt = *opt;
  b->stream = (hipStream_t)b->opt.stream;
  b->G = n_graphs;
  hipStream_t s = b->stream;
  // pinned staging for every host copy of the batch's passes (histograms
  // at the largest batch graph size)
  const size_t Gp = (size_t)n_graphs + 1;
  const size_t o_off = 0, o_nnz = align_up(Gp * 4, 256), o_stat = o_nnz + 256;
  const size_t o_bound = o_stat + align_up(Gp * 4, 256);
  const size_t o_root = o_bound + align_up(Gp * 8, 256);
  const size_t o_hist = o_root + align_up(Gp * 8, 256);
  const size_t stage = o_hist + align_up(Gp * (CC_BATCH_MAXN + 2) * 8, 256);
  if (!batch_res_take(dev, stage, &b->res)) return fail(CC_ERR_OUT_OF_MEMORY);
  char *hs = b->res.h_stage;
  b->s_off = (int32_t *)(hs + o_off);
  b->s_nnz = (int32_t *)(hs + o_nnz);
  b->s_stat = (unsigned int *)(hs + o_stat);
  b->s_bound = (long long *)(hs + o_bound);
  b->s_root = (long long *)(hs + o_root);
  b->s_hist = (unsigned long long *)(hs + o_hist);
  b->h_ctl = (CcCtl *)b->res.h_ctl;
  b->ev0 = b->res.ev[0];
  b->ev1 = b->res.ev[1];
  for (int i = 0; i < 4; ++i) b->evp[i] = b->res.ev[2 + i];
  // sizes and offsets are needed on the host (a device CSR is read on the
  // caller's stream, after whatever wrote it)
  int32_t *off = b->s_off;
  int32_t nnz = 0;
  if (flags & CC_INPUT_DEVICE) {
    if (hipMemcpyAsync(off, graph_vtx_off, Gp * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return fail(CC_ERR_DEVICE);
  } else {
    std::memcpy(off, graph_vtx_off, Gp * 4);
  }
  if (off[0] != 0) return fail(CC_ERR_INVALID_ARG);
  int max_n = 0;
  for (int g = 0; g < n_graphs; ++g) {
    const int ng = off[g + 1] - off[g];
    if (ng < 0) return fail(CC_ERR_INVALID_ARG);
    if (ng > CC_BATCH_MAXN) return fail(CC_ERR_TOO_LARGE);
    max_n = std::max(max_n, ng);
  }
  const int32_t N = off[n_graphs];
  if (n_graphs > 0) {
    if (flags & CC_INPUT_DEVICE) {
      if (hipMemcpyAsync(b->s_nnz, row_ptr + N, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess)
        return fail(CC_ERR_DEVICE);
      nnz = *b->s_nnz;
    } else {
      nnz = row_ptr[N];
      if (row_ptr[0] != 0) return fail(CC_ERR_NOT_SIMPLE);
    }
    if (nnz < 0) return fail(CC_ERR_NOT_SIMPLE);
    if (nnz > 0 && !col_idx) return fail(CC_ERR_INVALID_ARG);
  }
  b->N = N;
  b->W = max_n <= 64 ? 1 : max_n <= 128 ? 2 : 4;
  b->max_n = max_n;
  b->vtx_off.assign(off, off + Gp);
  const size_t Np = (size_t)std::max(N, 1);
  const size_t sz_off = align_up(Gp * 4, 256), sz_roff = align_up(Gp * 8, 256);
  const size_t sz_adj = align_up(Np * b->W * 8, 256), sz_vec = align_up(Np * 4, 256);
  const size_t sz_st = align_up(Gp * 4, 256), sz_bd = align_up(Gp * 8, 256);
  const size_t blob = sz_off + sz_roff + 2 * sz_adj + 2 * sz_vec + sz_st + sz_bd +
                      align_up(sizeof(CcCtl), 256);
  if (!batch_res_blob(b->res, blob)) return fail(CC_ERR_OUT_OF_MEMORY);
  b->d_blob = b->res.d_blob;
  char *p = (char *)b->d_blob;
  b->d_vtx_off = (int *)p; p += sz_off;
  b->d_root_off = (long long *)p; p += sz_roff;
  b->d_adj = (unsigned long long *)p; p += sz_adj;
  b->d_adj_orig = (unsigned long long *)p; p += sz_adj;
  b->d_perm = (int *)p; p += sz_vec;
  b->d_label = (int *)p; p += sz_vec;
  b->d_status = (unsigned int *)p; p += sz_st;
  b->d_bound = (long long *)p; p += sz_bd;
  b->d_ctl = (CcCtl *)p;
  b->root_off.assign(Gp, 0);
  if (n_graphs == 0) {
    *out = b;
    return CC_OK;
  }
  const int *d_rp = row_ptr, *d_ci = col_idx;
  void *tmp = nullptr;
  if (hipMemcpyAsync(b->d_vtx_off, off, Gp * 4, hipMemcpyHostToDevice, s) != hipSuccess)
    return fail(CC_ERR_DEVICE);
  if (!(flags & CC_INPUT_DEVICE)) {
    const size_t rb = align_up(((size_t)N + 1) * 4, 256);
    if (hipMallocAsync(&tmp, rb + (size_t)std::max(nnz, 1) * 4, s) != hipSuccess)
      return fail(CC_ERR_OUT_OF_MEMORY);
    if (hipMemcpyAsync(tmp, row_ptr, ((size_t)N + 1) * 4, hipMemcpyHostToDevice, s) != hipSuccess ||
        (nnz > 0 && hipMemcpyAsync((char *)tmp + rb, col_idx, (size_t)nnz * 4,
                                   hipMemcpyHostToDevice, s) != hipSuccess)) {
      (void)hipFreeAsync(tmp, s);
      (void)hipStreamSynchronize(s);
      return fail(CC_ERR_DEVICE);
    }
    d_rp = (const int *)tmp;
    d_ci = (const int *)((char *)tmp + rb);
  }
  hipError_t e = cc_launch_ingest(b->W, n_graphs, b->d_vtx_off, 0, d_rp, d_ci, b->d_adj,
                                  b->d_adj_orig, b->d_perm, b->d_label, b->d_status, b->d_bound,
                                  nullptr, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->s_stat, b->d_status, (size_t)n_graphs * 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->s_bound, b->d_bound, (size_t)n_graphs * 8, hipMemcpyDeviceToHost, s);
  if (tmp) (void)hipFreeAsync(tmp, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(hip_err(e));
  long long *root = b->s_root;
  root[0] = 0;
  for (int g = 0; g < n_graphs; ++g) {
    const unsigned int stg = b->s_stat[g];
    if ((stg & 0xffu) != 0u || !(stg & 0x100u)) return fail(CC_ERR_NOT_SIMPLE);
    b->max_deg = std::max(b->max_deg, (int)(stg >> 16));
    root[g + 1] = root[g] + b->s_bound[g];
  }
  b->root_off.assign(root, root + Gp);
  // (ordered before every later use of the root offsets on this stream;
  // the staging stays untouched until the batch is released)
  if (hipMemcpyAsync(b->d_root_off, root, Gp * 8, hipMemcpyHostToDevice, s) != hipSuccess)
    return fail(CC_ERR_DEVICE);
  *out = b;
  return CC_OK;
}

cc_status cc_histogram_batch_mode(cc_batch *b, int64_t *hists, const int64_t *hist_off,
                                  int32_t mode) {
  if (!b || (b->G > 0 && (!hists || !hist_off))) return CC_ERR_INVALID_ARG;
  if (mode != CC_BATCH_PERSISTENT && mode != CC_BATCH_PER_GRAPH) return CC_ERR_INVALID_ARG;
  for (int g = 0; g < b->G; ++g)
    if (hist_off[g] < 0) return CC_ERR_INVALID_ARG;
  if (hipSetDevice(b->device) != hipSuccess) return CC_ERR_DEVICE;
  const int G = b->G;
  b->info = cc_run_info{};
  if (G == 0) return CC_OK;
  hipStream_t s = b->stream;
  const int W = b->W;
  const int dstride = b->max_n + 2;
  const unsigned long long rcap = std::max<long long>(b->root_off[G], 1);
  int waves_per_cu = b->opt.dfs_waves_per_cu > 0 ? b->opt.dfs_waves_per_cu : 24;
  waves_per_cu = std::min(std::max(waves_per_cu, 4), 32);
  waves_per_cu = std::min(waves_per_cu, 4 * cc_dfs_blocks_per_cu(W, false, true));
  const bool per_graph = mode == CC_BATCH_PER_GRAPH;
  // both forms launch the depth-first kernel on the same full grid
  const int want_waves = std::max(4, (b->dev.cus * waves_per_cu) / 4 * 4);
  const int64_t budget = b->opt.frontier_budget_bytes > 0 ? b->opt.frontier_budget_bytes
                                                          : kDefaultBudget;
  // workspace: root slots (X words, end vertices, graph id), per-graph
  // histograms, and the depth-first stacks in the rest of the budget
  const size_t roots_b = align_up(rcap * W * 8, 256) + align_up(rcap * 2, 256) +
                         align_up(rcap * 4, 256);
  const size_t hist_b = align_up((size_t)G * dstride * 8, 256);
  const size_t stack_b = (size_t)std::max<int64_t>(budget / 2, (int64_t)64 << 20);
  char *arena = nullptr;
  CC_TRY(hipMallocAsync((void **)&arena, roots_b + hist_b + stack_b, s));
  BatchDev bt{};
  bt.vtx_off = b->d_vtx_off;
  bt.adj = b->d_adj;
  bt.perm = b->d_perm;
  bt.root_off = b->d_root_off;
  bt.rX = (unsigned long long *)arena;
  bt.rvv = (unsigned short *)(arena + align_up(rcap * W * 8, 256));
  bt.rgid = (unsigned int *)(arena + align_up(rcap * W * 8, 256) + align_up(rcap * 2, 256));
  bt.rcap = rcap;
  bt.hist = (unsigned long long *)(arena + roots_b);
  bt.hist_stride = dstride;
  bt.n_graphs = G;
  DfsWork wk{};
  const int nw = carve_dfs(arena + roots_b + hist_b, stack_b, W, false, want_waves, &wk, true);
  if (nw < 4) {
    (void)hipFreeAsync(arena, s);
    return CC_ERR_OUT_OF_MEMORY;
  }
  if (b->opt.dfs_donate_min > 0) wk.donate_min = b->opt.dfs_donate_min;
  wk.claim = b->opt.dfs_claim > 0 ? (b->opt.dfs_claim + CC_CHUNK - 1) / CC_CHUNK * CC_CHUNK : 0;
  const unsigned long long idle_timeout =
      (unsigned long long)(kIdleTimeoutSeconds * (double)b->dev.clock_hz);
  GraphDev gd{b->d_adj, b->d_adj_orig, b->d_perm, b->max_n};
  CcCtl *ctl = b->d_ctl;
  hipError_t e = hipSuccess;
  auto chk = [&](hipError_t x) {
    if (x != hipSuccess && e == hipSuccess) e = x;
  };
  // CC_PROFILE (persistent form): HIP events on this stream around stage
  // one and around the depth-first kernel
  const bool prof = (b->opt.flags & CC_PROFILE) != 0 && !per_graph;
  if (prof)
    for (hipEvent_t &ev : b->evp)
      if (!ev) chk(hipEventCreate(&ev));
  chk(hipEventRecord(b->ev0, s));
  chk(cc_launch_zero(ctl, sizeof(CcCtl), s));
  chk(cc_launch_zero(bt.hist, hist_b, s));
  int launches = 0;
  if (!per_graph) {
    // one launch for stage one of every graph, one persistent depth-first
    // launch over all their initial triplets
    bt.g0 = 0;
    if (prof) chk(hipEventRecord(b->evp[0], s));
    chk(cc_launch_triplets_batch(W, bt, G, s));
    if (prof) chk(hipEventRecord(b->evp[1], s));
    bt.r0 = 0;
    bt.r1 = (unsigned long long)b->root_off[G];
    chk(cc_launch_dfs_prepare(ctl, wk, b->max_n, false, s));
    if (prof) chk(hipEventRecord(b->evp[2], s));
    chk(cc_launch_dfs_batch(W, gd, ctl, wk, bt, nw / 4, idle_timeout, s));
    if (prof) chk(hipEventRecord(b->evp[3], s));
    launches = 3;
  } else {
    // the same kernels, one graph at a time
    for (int g = 0; g < G && e == hipSuccess; ++g) {
      bt.g0 = g;
      chk(cc_launch_triplets_batch(W, bt, 1, s));
      bt.r0 = (unsigned long long)b->root_off[g];
      bt.r1 = (unsigned long long)b->root_off[g + 1];
      chk(cc_launch_dfs_prepare(ctl, wk, b->max_n, false, s));
      chk(cc_launch_dfs_batch(W, gd, ctl, wk, bt, nw / 4, idle_timeout, s));
      launches += 3;
    }
  }
  chk(hipEventRecord(b->ev1, s));
  unsigned long long *hh = b->s_hist;  // pinned, G * dstride words
  chk(hipMemcpyAsync(hh, bt.hist, (size_t)G * dstride * 8, hipMemcpyDeviceToHost, s));
  const size_t tail = offsetof(CcCtl, peak);  // a batch reads only the scalars
  chk(hipMemcpyAsync((char *)b->h_ctl + tail, (char *)ctl + tail, sizeof(CcCtl) - tail,
                     hipMemcpyDeviceToHost, s));
  chk(hipFreeAsync(arena, s));
  chk(hipStreamSynchronize(s));
  if (e != hipSuccess) return hip_err(e);
  int64_t cycles = 0, paths = 0;
  for (int g = 0; g < G; ++g) {
    const int ng = b->vtx_off[g + 1] - b->vtx_off[g];
    int64_t *dst = hists + hist_off[g];
    for (int k = 0; k <= ng; ++k) {
      dst[k] = (int64_t)hh[(size_t)g * dstride + k];
      cycles += (int64_t)hh[(size_t)g * dstride + k];
    }
  }
  paths = (int64_t)b->h_ctl->dfs_lanes;
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, b->ev0, b->ev1);
  b->info.cycles = cycles;
  b->info.paths = paths;
  b->info.levels_launched = launches;
  b->info.gpu_ms = ms;
  if (prof) {
    float a = 0.f, c = 0.f;
    (void)hipEventElapsedTime(&a, b->evp[0], b->evp[1]);
    (void)hipEventElapsedTime(&c, b->evp[2], b->evp[3]);
    b->info.stage1_ms = a;
    b->info.dfs_ms = c;
  }
  b->info.device_diag = (int64_t)b->h_ctl->diag;
  dfs_stats(*b->h_ctl, &b->info);
  if (b->h_ctl->status & (CC_DEV_CORRUPT | CC_DEV_LOST)) return CC_ERR_INTERNAL;
  if (b->h_ctl->status & CC_DEV_STACK_FULL) return CC_ERR_OUT_OF_MEMORY;
  return CC_OK;
}

cc_status cc_histogram_batch(cc_batch *b, int64_t *hists, const int64_t *hist_off) {
  return cc_histogram_batch_mode(b, hists, hist_off, CC_BATCH_PERSISTENT);
}

cc_status cc_batch_last_run(cc_batch *b, cc_run_info *info) {
  if (!b || !info) return CC_ERR_INVALID_ARG;
  *info = b->info;
  return CC_OK;
}

cc_status cc_batch_labels(cc_batch *b, int32_t *labels) {
  if (!b || !labels) return CC_ERR_INVALID_ARG;
  if (b->N == 0) return CC_OK;
  if (hipSetDevice(b->device) != hipSuccess ||
      hipMemcpyAsync(labels, b->d_label, (size_t)b->N * 4, hipMemcpyDeviceToHost, b->stream) !=
          hipSuccess ||
      hipStreamSynchronize(b->stream) != hipSuccess)
    return CC_ERR_DEVICE;
  return CC_OK;
}

}  // extern "C"


// ---------------------------------------------------- no-allocation variant
// cc_histogram_noalloc: the count-only run of cc_prepare + cc_histogram for
// callers that cannot allocate.  Every buffer the kernels need beyond the
// caller's inputs and output (control block, bitsets, labels, the two
// frontier buffers, the depth-first stacks and mailboxes) is carved from
// `scratch`, a file-scope device array of kScratchBytes that each GPU holds
// from module load until the process ends.  In host code the array's name
// is only a stand-in: its device address comes from hipGetSymbolAddress,
// once per device, and only that address is handed to kernels and copies.
// No call here allocates: no hipMalloc/hipFree, no pinned host memory (the
// host learns the ingest's answer and the run's status by small copies into
// its own stack and a stream synchronisation), no library routine that
// allocates.  Every call on a device uses that device's one array, so calls
// that overlap on one device race; each call re-zeroes what must start at
// zero (the control block, the depth-first mailboxes).
namespace {
constexpr size_t kScratchBytes = 64ull << 20;
constexpr size_t kScratchFrontier = 24ull << 20;  // both frontier buffers together
}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_scratch_mu;
void *g_scratch_ptr[64];

// The device address of `scratch` on device dev (dev current).
cc_status scratch_address(int dev, char **out) {
  if (dev < 0 || dev >= 64) return CC_ERR_NO_DEVICE;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return CC_ERR_DEVICE;
    g_scratch_ptr[dev] = p;
  }
  *out = (char *)g_scratch_ptr[dev];
  return CC_OK;
}

}  // namespace

extern "C" cc_status cc_histogram_noalloc(int32_t n, const int32_t *row_ptr,
                                          const int32_t *col_idx, int64_t *hist,
                                          int32_t hist_len, void *stream) {
  if (n < 0 || !hist || hist_len < n + 1 || (n > 0 && (!row_ptr || !col_idx)))
    return CC_ERR_INVALID_ARG;
  if (n > CC_MAX_VERTICES) return CC_ERR_TOO_LARGE;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return CC_ERR_NO_DEVICE;
  DeviceInfo di;
  cc_status st = device_info(dev, &di);
  if (st != CC_OK) return st;
  char *base = nullptr;
  st = scratch_address(dev, &base);
  if (st != CC_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  const int W = words_for(n);
  // fixed part of the scratch: control block, bitsets, labels, ingest answer
  size_t off = 0;
  auto take = [&](size_t b) {
    char *q = base + off;
    off = align_up(off + b, 256);
    return q;
  };
  CcCtl *ctl = (CcCtl *)take(sizeof(CcCtl));
  unsigned long long *adj = (unsigned long long *)take((size_t)CC_MAXN * CC_MAXN / 8);
  unsigned long long *adj_orig = (unsigned long long *)take((size_t)CC_MAXN * CC_MAXN / 8);
  int *perm = (int *)take((size_t)CC_MAXN * 4);
  int *label = (int *)take((size_t)CC_MAXN * 4);
  unsigned int *status = (unsigned int *)take(256);
  long long *pairs = (long long *)((char *)status + 8);
  hipError_t e = hipSuccess;
  auto chk = [&](hipError_t x) {
    if (x != hipSuccess && e == hipSuccess) e = x;
  };
  // ingest: validation, labelling, bitsets; its answer (status word, then
  // the sum over vertices of C(deg, 2)) comes back by a copy
  unsigned long long answer[2] = {0ull, 0ull};
  if (n > 0) {
    chk(cc_launch_ingest(W, 1, nullptr, n, row_ptr, col_idx, adj, adj_orig, perm, label, status,
                         pairs, nullptr, s));
    chk(hipMemcpyAsync(answer, status, sizeof(answer), hipMemcpyDeviceToHost, s));
    chk(hipStreamSynchronize(s));
    if (e != hipSuccess) return hip_err(e);
    const unsigned stv = (unsigned)answer[0];
    if ((stv & 0xffu) != 0u || !(stv & 0x100u)) return CC_ERR_NOT_SIMPLE;
  }
  if (n < 3) {
    chk(cc_launch_zero(hist, (size_t)hist_len * 8, s));
    chk(hipStreamSynchronize(s));
    return hip_err(e);
  }
  const int max_deg = (int)((unsigned)answer[0] >> 16);
  const int64_t npairs = (int64_t)answer[1];
  // the frontier buffers: every initial triplet (at most sum C(deg, 2))
  // must fit, dealt round-robin over the shards
  const size_t per_unit = 2 * ((size_t)W * 8 + vv_bytes(W));
  const unsigned long long min_cap_s =
      (unsigned long long)std::min<int64_t>(npairs, choose3(n)) / CC_SHARDS + CC_CHUNK;
  const unsigned long long cap_s =
      ((unsigned long long)(kScratchFrontier / per_unit / CC_SHARDS)) & ~63ull;
  if (cap_s < min_cap_s) return CC_ERR_OUT_OF_MEMORY;  // more initial triplets than the scratch holds
  const size_t buf_bytes = align_up(frontier_bytes(cap_s, W, false), 256);
  LevelBufs lb{};
  lb.f[0] = carve_frontier(take(buf_bytes), cap_s, W, false);
  lb.f[1] = carve_frontier(take(buf_bytes), cap_s, W, false);
  if (off >= kScratchBytes) return CC_ERR_OUT_OF_MEMORY;
  // the rest: the depth-first workspace
  DfsWork wk{};
  const int wpc = std::min(24, 4 * cc_dfs_blocks_per_cu(W, false, false));
  const int nw = carve_dfs(base + off, kScratchBytes - off, W, false,
                           std::max(4, di.cus * wpc / 4 * 4), &wk);
  if (nw < 4) return CC_ERR_OUT_OF_MEMORY;
  const unsigned long long idle_timeout =
      (unsigned long long)(kIdleTimeoutSeconds * (double)di.clock_hz);
  GraphDev gd{adj, adj_orig, perm, n};
  const OutDev out{};
  const int maxc = std::max(1, max_deg - 1);
  const int bfs_blocks = di.cus * std::min(cc_step_blocks_per_cu(W, false), kStepBlocksPerCu);
  const size_t head_lds = head_dyn_lds(W, false, di.lds_block);
  // the head zeroes the control block, runs stage one and the leading
  // levels; every later step launch returns at once after the loop is over
  // (the host has no mapped word to stop early, so it queues all n - 2)
  chk(cc_launch_head(W, false, gd, ctl, lb, out, -1, head_lds, nullptr, true, RootRange{}, s));
  for (int launch = 1; launch < n - 1 && e == hipSuccess; ++launch)
    chk(cc_launch_step(W, false, gd, ctl, lb, out, launch, -1, maxc, true, bfs_blocks, nullptr,
                       s));
  // the depth-first continuation returns at once if nothing was handed over
  chk(cc_launch_dfs_prepare(ctl, wk, n, false, s));
  chk(cc_launch_dfs(W, false, gd, ctl, lb.f[0], lb.f[1], wk, out,
                    dev_field(ctl, offsetof(CcCtl, hist_sh)), CC_HSLOTS, true, nw / 4,
                    idle_timeout, s));
  chk(cc_launch_finalize(ctl, out, n, false, s));
  // the histogram (n + 1 entries) into the caller's array, zeros after it
  chk(hipMemcpyAsync(hist, ctl->hist, (size_t)(n + 1) * 8, hipMemcpyDeviceToDevice, s));
  if (hist_len > n + 1) chk(cc_launch_zero(hist + n + 1, (size_t)(hist_len - n - 1) * 8, s));
  unsigned int dstat = 0u;
  chk(hipMemcpyAsync(&dstat, &ctl->status, 4, hipMemcpyDeviceToHost, s));
  chk(hipStreamSynchronize(s));
  if (e != hipSuccess) return hip_err(e);
  if (dstat & (CC_DEV_CORRUPT | CC_DEV_LOST)) return CC_ERR_INTERNAL;
  if (dstat & CC_DEV_STACK_FULL) return CC_ERR_OUT_OF_MEMORY;
  return CC_OK;
}

// ------------------------------------------------------------------ serving
// A request loop over the batched kernels.  Requests (one graph each) are
// copied in at submission; a dispatcher thread admits pending requests into
// a free device slot by the policy of cc_serve_policy.h, packs them, and
// launches ingest -> stage one -> one persistent depth-first launch on that
// slot's stream, sized to its share of the CUs.  Several slots run at once,
// so requests that arrive while others are on the GPU start as soon as a
// slot frees up and their work overlaps on the device.  Completion is
// detected with an event per slot; no launch waits on the host.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <thread>
#include <unordered_map>

#include "cc_serve_policy.h"

namespace {

using Clock = std::chrono::steady_clock;

struct ServeReq {
  int64_t id = 0;
  int32_t n = 0;
  std::vector<int32_t> rp, ci;
  ccserve::Cost cost;
  Clock::time_point t_submit, t_start, t_done;
  int state = 0;  // 0 pending, 1 on the device, 2 done
  cc_status status = CC_OK;
  std::vector<int64_t> hist;
};

// per-length histogram slots of a served graph (at most CC_BATCH_MAXN vertices)
constexpr int kServeSlots = CC_BATCH_MAXN + 2;

struct ServeSlot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  bool busy = false;
  std::vector<ServeReq *> reqs;
  void *dev = nullptr;   // one allocation for all device buffers
  void *host = nullptr;  // one pinned allocation for staging
  int *d_vtx_off = nullptr, *d_rp = nullptr, *d_ci = nullptr;
  long long *d_root_off = nullptr, *d_bound = nullptr;
  unsigned long long *d_adj = nullptr, *d_adj_orig = nullptr;
  int *d_perm = nullptr, *d_label = nullptr;
  unsigned int *d_status = nullptr;
  unsigned long long *rX = nullptr, *d_hist = nullptr;
  unsigned short *rvv = nullptr;
  unsigned int *rgid = nullptr;
  CcCtl *d_ctl = nullptr;
  char *d_work = nullptr;
  size_t work_bytes = 0;
  int *h_vtx_off = nullptr, *h_rp = nullptr, *h_ci = nullptr;
  long long *h_root_off = nullptr;
  unsigned long long *h_hist = nullptr;
  unsigned int *h_status = nullptr;
  unsigned int *h_ctl_status = nullptr;
};

}  // namespace

struct cc_server {
  int device = 0;
  DeviceInfo dev{};
  cc_server_options opt{};
  ccserve::Capacity cap;
  std::mutex mu;
  std::condition_variable cv;       // wakes the dispatcher
  std::condition_variable done_cv;  // wakes waiters
  std::deque<std::pair<ServeReq *, ccserve::Cost>> pending;
  std::unordered_map<int64_t, ServeReq *> reqs;
  std::vector<ServeSlot> slots;
  std::thread th;
  bool stop = false;
  int64_t next_id = 1;
  int64_t batches = 0, completed = 0, rejected = 0, max_batch = 0;
  double busy_slot_ms = 0.0;
};

namespace {

size_t a256(size_t x) { return align_up(x, 256); }

cc_status slot_alloc(cc_server *sv, ServeSlot &sl) {
  const ccserve::Capacity &c = sv->cap;
  const size_t G = (size_t)c.graphs, V = (size_t)c.vertices + CC_BATCH_MAXN, E = (size_t)c.entries,
               R = (size_t)c.roots;
  const size_t dev_fixed = a256((G + 1) * 4) + a256((V + 1) * 4) + a256(E * 4) +
                           2 * a256((G + 1) * 8) + 2 * a256(V * 4 * 8) + 2 * a256(V * 4) +
                           a256(G * 4) + a256(R * 4 * 8) + a256(R * 2) + a256(R * 4) +
                           a256(G * kServeSlots * 8) + a256(sizeof(CcCtl));
  sl.work_bytes = (size_t)sv->opt.slot_work_bytes;
  if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess)
    return CC_ERR_DEVICE;
  if (hipMalloc(&sl.dev, dev_fixed + sl.work_bytes) != hipSuccess) return CC_ERR_OUT_OF_MEMORY;
  char *p = (char *)sl.dev;
  auto take = [&](size_t b) {
    char *q = p;
    p += a256(b);
    return q;
  };
  sl.d_vtx_off = (int *)take((G + 1) * 4);
  sl.d_rp = (int *)take((V + 1) * 4);
  sl.d_ci = (int *)take(E * 4);
  sl.d_root_off = (long long *)take((G + 1) * 8);
  sl.d_bound = (long long *)take((G + 1) * 8);
  sl.d_adj = (unsigned long long *)take(V * 4 * 8);  // up to four words a row
  sl.d_adj_orig = (unsigned long long *)take(V * 4 * 8);
  sl.d_perm = (int *)take(V * 4);
  sl.d_label = (int *)take(V * 4);
  sl.d_status = (unsigned int *)take(G * 4);
  sl.rX = (unsigned long long *)take(R * 4 * 8);
  sl.rvv = (unsigned short *)take(R * 2);
  sl.rgid = (unsigned int *)take(R * 4);
  sl.d_hist = (unsigned long long *)take(G * kServeSlots * 8);
  sl.d_ctl = (CcCtl *)take(sizeof(CcCtl));
  sl.d_work = p;
  const size_t host_b = a256((G + 1) * 4) + a256((V + 1) * 4) + a256(E * 4) + a256((G + 1) * 8) +
                        a256(G * kServeSlots * 8) + a256(G * 4) + a256(4);
  if (hipHostMalloc(&sl.host, host_b, hipHostMallocDefault) != hipSuccess)
    return CC_ERR_OUT_OF_MEMORY;
  char *h = (char *)sl.host;
  auto htake = [&](size_t b) {
    char *q = h;
    h += a256(b);
    return q;
  };
  sl.h_vtx_off = (int *)htake((G + 1) * 4);
  sl.h_rp = (int *)htake((V + 1) * 4);
  sl.h_ci = (int *)htake(E * 4);
  sl.h_root_off = (long long *)htake((G + 1) * 8);
  sl.h_hist = (unsigned long long *)htake(G * kServeSlots * 8);
  sl.h_status = (unsigned int *)htake(G * 4);
  sl.h_ctl_status = (unsigned int *)htake(4);
  return CC_OK;
}

// Packs the admitted requests into the slot's staging area and enqueues the
// whole batch on the slot's stream.  The slot and its requests belong to the
// dispatcher while the slot is busy, so this runs without the server lock.
hipError_t slot_launch(cc_server *sv, ServeSlot &sl, const std::vector<ServeReq *> &rs) {
  const int G = (int)rs.size();
  int max_n = 0, max_deg = 0;
  long long roots = 0;
  int32_t v = 0, e = 0;
  sl.h_vtx_off[0] = 0;
  sl.h_rp[0] = 0;
  sl.h_root_off[0] = 0;
  for (int g = 0; g < G; ++g) {
    const ServeReq *r = rs[g];
    max_n = std::max(max_n, r->n);
    for (int32_t i = 0; i < r->n; ++i) {
      sl.h_rp[v + i + 1] = e + r->rp[i + 1];
      max_deg = std::max(max_deg, r->rp[i + 1] - r->rp[i]);
    }
    // an id outside the graph becomes -1, which ingest rejects as not simple
    for (size_t i = 0; i < r->ci.size(); ++i) {
      const int32_t c = r->ci[i];
      sl.h_ci[e + i] = (c >= 0 && c < r->n) ? c + v : -1;
    }
    v += r->n;
    e += (int32_t)r->ci.size();
    roots += r->cost.roots;
    sl.h_vtx_off[g + 1] = v;
    sl.h_root_off[g + 1] = roots;
  }
  const int W = max_n <= 64 ? 1 : max_n <= 128 ? 2 : 4;
  const int wpc = std::min(std::max(4, sv->opt.dfs_waves_per_cu),
                           4 * cc_dfs_blocks_per_cu(W, false, true));
  const int waves = std::max(4, sv->dev.cus * wpc / std::max(1, (int)sv->slots.size()) / 4 * 4);
  DfsWork wk{};
  const int nw = carve_dfs(sl.d_work, sl.work_bytes, W, false, waves, &wk, true);
  if (nw < 4) return hipErrorOutOfMemory;
  hipStream_t s = sl.stream;
  hipError_t err = hipSuccess;
  auto chk = [&](hipError_t x) {
    if (x != hipSuccess && err == hipSuccess) err = x;
  };
  chk(hipMemcpyAsync(sl.d_vtx_off, sl.h_vtx_off, (size_t)(G + 1) * 4, hipMemcpyHostToDevice, s));
  chk(hipMemcpyAsync(sl.d_rp, sl.h_rp, (size_t)(v + 1) * 4, hipMemcpyHostToDevice, s));
  if (e > 0) chk(hipMemcpyAsync(sl.d_ci, sl.h_ci, (size_t)e * 4, hipMemcpyHostToDevice, s));
  chk(hipMemcpyAsync(sl.d_root_off, sl.h_root_off, (size_t)(G + 1) * 8, hipMemcpyHostToDevice, s));
  chk(cc_launch_ingest(W, G, sl.d_vtx_off, 0, sl.d_rp, sl.d_ci, sl.d_adj, sl.d_adj_orig, sl.d_perm,
                       sl.d_label, sl.d_status, sl.d_bound, nullptr, s));
  chk(cc_launch_zero(sl.d_ctl, sizeof(CcCtl), s));
  chk(cc_launch_zero(sl.d_hist, (size_t)G * kServeSlots * 8, s));
  BatchDev bt{};
  bt.vtx_off = sl.d_vtx_off;
  bt.adj = sl.d_adj;
  bt.perm = sl.d_perm;
  bt.root_off = sl.d_root_off;
  bt.rX = sl.rX;
  bt.rvv = sl.rvv;
  bt.rgid = sl.rgid;
  bt.rcap = (unsigned long long)sv->cap.roots;
  bt.r0 = 0;
  bt.r1 = (unsigned long long)roots;
  bt.hist = sl.d_hist;
  bt.hist_stride = kServeSlots;
  bt.g0 = 0;
  bt.n_graphs = G;
  chk(cc_launch_triplets_batch(W, bt, G, s));
  GraphDev gd{sl.d_adj, sl.d_adj_orig, sl.d_perm, max_n};
  chk(cc_launch_dfs_prepare(sl.d_ctl, wk, max_n, false, s));
  chk(cc_launch_dfs_batch(W, gd, sl.d_ctl, wk, bt, nw / 4,
                          (unsigned long long)(kIdleTimeoutSeconds * (double)sv->dev.clock_hz), s));
  chk(hipMemcpyAsync(sl.h_hist, sl.d_hist, (size_t)G * kServeSlots * 8, hipMemcpyDeviceToHost, s));
  chk(hipMemcpyAsync(sl.h_status, sl.d_status, (size_t)G * 4, hipMemcpyDeviceToHost, s));
  chk(hipMemcpyAsync(sl.h_ctl_status, &sl.d_ctl->status, 4, hipMemcpyDeviceToHost, s));
  chk(hipEventRecord(sl.done, s));
  return err;
}

void slot_finish(cc_server *sv, ServeSlot &sl, hipError_t ev) {
  const Clock::time_point now = Clock::now();
  for (size_t g = 0; g < sl.reqs.size(); ++g) {
    ServeReq *r = sl.reqs[g];
    if (ev != hipSuccess) {
      r->status = ev == hipErrorOutOfMemory ? CC_ERR_OUT_OF_MEMORY : CC_ERR_DEVICE;
    } else if (*sl.h_ctl_status & (CC_DEV_CORRUPT | CC_DEV_LOST)) {
      r->status = CC_ERR_INTERNAL;  // a consistency check failed: the batch is discarded
    } else if (*sl.h_ctl_status & CC_DEV_STACK_FULL) {
      r->status = CC_ERR_OUT_OF_MEMORY;  // a depth-first stack ran out: counts incomplete
    } else if ((sl.h_status[g] & 0xffu) != 0u || !(sl.h_status[g] & 0x100u)) {
      r->status = CC_ERR_NOT_SIMPLE;
    } else {
      r->status = CC_OK;
      r->hist.assign((size_t)r->n + 1, 0);
      for (int k = 0; k <= r->n; ++k) r->hist[k] = (int64_t)sl.h_hist[g * kServeSlots + k];
    }
    r->t_done = now;
    r->state = 2;
    sv->completed++;
  }
  sl.reqs.clear();
  sl.busy = false;
}

void dispatcher(cc_server *sv) {
  (void)hipSetDevice(sv->device);
  std::unique_lock<std::mutex> lk(sv->mu);
  while (true) {
    bool any_busy = false, progressed = false;
    for (ServeSlot &sl : sv->slots) {
      if (!sl.busy) continue;
      const hipError_t q = hipEventQuery(sl.done);
      if (q == hipErrorNotReady) {
        any_busy = true;
        continue;
      }
      slot_finish(sv, sl, q);
      progressed = true;
    }
    if (progressed) sv->done_cv.notify_all();
    for (ServeSlot &sl : sv->slots) {
      if (sl.busy || sv->pending.empty()) continue;
      std::vector<ServeReq *> rs = ccserve::admit(sv->pending, sv->cap);
      if (rs.empty()) break;  // cannot happen: oversize requests are rejected at submit
      const Clock::time_point now = Clock::now();
      for (ServeReq *r : rs) {
        r->state = 1;
        r->t_start = now;
      }
      sl.reqs = rs;
      sl.busy = true;
      any_busy = true;
      sv->batches++;
      sv->max_batch = std::max<int64_t>(sv->max_batch, (int64_t)rs.size());
      lk.unlock();
      const hipError_t e = slot_launch(sv, sl, rs);
      lk.lock();
      if (e != hipSuccess) {
        (void)hipStreamSynchronize(sl.stream);
        slot_finish(sv, sl, e);
        sv->done_cv.notify_all();
      }
    }
    if (sv->stop && sv->pending.empty() && !any_busy) break;
    sv->cv.wait_for(lk, std::chrono::microseconds(any_busy ? 20 : 200));
  }
}

}  // namespace

extern "C" {

void cc_server_destroy(cc_server *sv) {
  if (!sv) return;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
  }
  sv->cv.notify_all();
  if (sv->th.joinable()) sv->th.join();
  (void)hipSetDevice(sv->device);
  for (ServeSlot &sl : sv->slots) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    if (sl.dev) (void)hipFree(sl.dev);
    if (sl.host) (void)hipHostFree(sl.host);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
  }
  for (auto &kv : sv->reqs) delete kv.second;
  delete sv;
}

cc_status cc_server_create(const cc_server_options *opt, cc_server **out) {
  if (!out) return CC_ERR_INVALID_ARG;
  *out = nullptr;
  cc_server_options o{};
  if (opt) o = *opt;
  if (o.slots < 0 || o.max_batch_graphs < 0 || o.slot_root_slots < 0 || o.slot_work_bytes < 0 ||
      o.dfs_waves_per_cu < 0)
    return CC_ERR_INVALID_ARG;
  if (o.slots == 0) o.slots = 4;
  if (o.max_batch_graphs == 0) o.max_batch_graphs = 256;
  if (o.slot_root_slots == 0) o.slot_root_slots = 1 << 22;
  if (o.slot_work_bytes == 0) o.slot_work_bytes = 256ll << 20;
  if (o.dfs_waves_per_cu == 0) o.dfs_waves_per_cu = 16;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return CC_ERR_NO_DEVICE;
  DeviceInfo di;
  cc_status st = device_info(dev, &di);
  if (st != CC_OK) return st;
  cc_server *sv = new cc_server();
  sv->device = dev;
  sv->dev = di;
  sv->opt = o;
  sv->cap.graphs = o.max_batch_graphs;
  sv->cap.vertices = (int64_t)o.max_batch_graphs * CC_BATCH_MAXN;
  sv->cap.entries = std::max<int64_t>((int64_t)o.max_batch_graphs * 1024, 1 << 20);
  sv->cap.roots = o.slot_root_slots;
  sv->slots.resize((size_t)o.slots);
  for (ServeSlot &sl : sv->slots) {
    st = slot_alloc(sv, sl);
    if (st != CC_OK) {
      cc_server_destroy(sv);
      return st;
    }
  }
  sv->th = std::thread(dispatcher, sv);
  *out = sv;
  return CC_OK;
}

cc_status cc_server_submit(cc_server *sv, int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                           int64_t *request_id) {
  if (!sv || !request_id || n < 0 || (n > 0 && !row_ptr)) return CC_ERR_INVALID_ARG;
  if (n > CC_MAX_BATCH_VERTICES) return CC_ERR_TOO_LARGE;
  const int32_t nnz = n > 0 ? row_ptr[n] : 0;
  if (n > 0 && (row_ptr[0] != 0 || nnz < 0 || (int64_t)nnz > (int64_t)n * (n - 1)))
    return CC_ERR_NOT_SIMPLE;
  if (nnz > 0 && !col_idx) return CC_ERR_INVALID_ARG;
  for (int32_t v = 0; v < n; ++v)
    if (row_ptr[v + 1] < row_ptr[v]) return CC_ERR_NOT_SIMPLE;
  ServeReq *r = new ServeReq();
  r->n = n;
  r->rp.assign(row_ptr, row_ptr + (n > 0 ? n + 1 : 0));
  if (n == 0) r->rp.assign(1, 0);
  r->ci.assign(col_idx, col_idx + nnz);
  r->cost = ccserve::cost_of(n, r->rp.data());
  r->t_submit = Clock::now();
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    r->id = sv->next_id++;
    *request_id = r->id;
    sv->reqs[r->id] = r;
    if (!ccserve::fits_empty(r->cost, sv->cap)) {
      r->status = CC_ERR_OUT_OF_MEMORY;  // larger than a whole slot
      r->state = 2;
      r->t_done = r->t_submit;
      sv->rejected++;
      sv->completed++;
    } else {
      sv->pending.emplace_back(r, r->cost);
    }
  }
  sv->cv.notify_all();
  return CC_OK;
}

cc_status cc_server_result(cc_server *sv, int64_t request_id, double timeout_s, int64_t *hist,
                           int32_t hist_len, double *latency_ms, cc_status *request_status) {
  if (!sv || !hist || hist_len < 1) return CC_ERR_INVALID_ARG;
  std::unique_lock<std::mutex> lk(sv->mu);
  auto it = sv->reqs.find(request_id);
  if (it == sv->reqs.end()) return CC_ERR_INVALID_ARG;
  ServeReq *r = it->second;
  if (hist_len < r->n + 1) return CC_ERR_INVALID_ARG;
  const auto deadline = Clock::now() + std::chrono::duration<double>(std::max(timeout_s, 0.0));
  while (r->state != 2) {
    if (sv->done_cv.wait_until(lk, deadline) == std::cv_status::timeout && r->state != 2)
      return CC_ERR_NOT_READY;
  }
  for (int k = 0; k < hist_len; ++k) hist[k] = k < (int)r->hist.size() ? r->hist[k] : 0;
  if (latency_ms)
    *latency_ms = std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count();
  if (request_status) *request_status = r->status;
  sv->reqs.erase(it);
  delete r;
  return CC_OK;
}

cc_status cc_server_stats(cc_server *sv, int64_t *stats, int32_t len) {
  if (!sv || !stats || len < 5) return CC_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(sv->mu);
  stats[0] = sv->completed;
  stats[1] = sv->batches;
  stats[2] = (int64_t)sv->pending.size();
  stats[3] = sv->rejected;
  stats[4] = sv->max_batch;
  return CC_OK;
}

}  // extern "C"
