/*
 * CPU oracle for chordless-cycle enumeration.  TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library.  It shares no code, header, table or helper with
 * the HIP path; the two only read the same generated CSR inputs.
 *
 * What it computes.  A chordless cycle of a finite undirected simple graph is
 * an induced subgraph that is a cycle (Section 1).  Its vertices are written
 * <v1, ..., vk> without repeating v1 (Section 2, with its footnote), and a
 * chord is an edge between two vertices of the path/cycle that is not part
 * of it (Section 2).
 *
 * How.  The sequential algorithm of Section 3 (Algorithm 1), in its
 * depth-first form, with the paper's own data layout: sorted adjacency
 * lists, adjacency tests by binary search (Section 4.2), explicit ordered
 * vertex paths.  The steps, in the paper's order:
 *   1. degree labelling (Section 2): repeatedly remove a vertex of minimum
 *      degree in the remaining graph; the i-th removed vertex gets label i
 *      (0-based here; ties broken by the smallest vertex id);
 *   2. stage one (Algorithm 1, triplet set T(G) and the triangles): for
 *      every u and pair x, y of its neighbours with l(u) < l(x) < l(y), a
 *      triangle <x,u,y> if (x,y) is an edge, else the chordless path
 *      <x,u,y>;
 *   3. expansion (Algorithm 1, the while loop): for a path <v1..vt> and each
 *      v in Adj(vt) with l(v) > l(v2) and v adjacent to none of v2..v(t-1):
 *      a cycle <v1..vt,v> if v is adjacent to v1, else the longer path.
 * The path-extension property of Section 2 guarantees that such a v never
 * repeats a path vertex; this is checked at run time and reported.
 *
 * Outputs per call: hist[k] = number of chordless cycles with k vertices,
 * front[t] = number of chordless paths with t vertices that were expanded
 * (front[3] = |T(G)|), the cycles themselves in path order (original ids),
 * and the labels.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum {
  ORC_OK = 0,
  ORC_ERR_INVALID_ARG = -1,
  ORC_ERR_NOT_SIMPLE = -2,
  ORC_ERR_OUT_OF_MEMORY = -5,
  ORC_ERR_INTERNAL = -7
};

/* ---------------------------------------------------------------- graph */
typedef struct {
  int32_t n;
  int32_t *start; /* n+1 offsets into nb */
  int32_t *nb;    /* sorted neighbour lists */
} orc_graph;

static int cmp_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}

/* Binary search for b in the sorted list of a (Section 4.2). */
static int adjacent(const orc_graph *g, int32_t a, int32_t b) {
  int32_t lo = g->start[a], hi = g->start[a + 1];
  while (lo < hi) {
    int32_t mid = lo + (hi - lo) / 2;
    int32_t w = g->nb[mid];
    if (w == b) return 1;
    if (w < b) lo = mid + 1; else hi = mid;
  }
  return 0;
}

/* Copies the CSR, sorts every list, and checks that the graph is simple and
 * undirected: offsets monotone, ids in range, no self-loop, no repeated
 * neighbour, every edge present in both directions. */
static int load_graph(int32_t n, const int32_t *rp, const int32_t *ci, orc_graph *g) {
  memset(g, 0, sizeof(*g));
  if (n < 0 || (n > 0 && (!rp))) return ORC_ERR_INVALID_ARG;
  g->n = n;
  g->start = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
  if (!g->start) return ORC_ERR_OUT_OF_MEMORY;
  if (n == 0) return ORC_OK;
  if (rp[0] != 0) return ORC_ERR_NOT_SIMPLE;
  for (int32_t v = 0; v < n; v++)
    if (rp[v + 1] < rp[v]) return ORC_ERR_NOT_SIMPLE;
  int32_t nnz = rp[n];
  if (nnz > 0 && !ci) return ORC_ERR_INVALID_ARG;
  g->nb = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
  if (!g->nb) return ORC_ERR_OUT_OF_MEMORY;
  memcpy(g->start, rp, sizeof(int32_t) * ((size_t)n + 1));
  if (nnz) memcpy(g->nb, ci, sizeof(int32_t) * (size_t)nnz);
  for (int32_t v = 0; v < n; v++) {
    int32_t a = g->start[v], b = g->start[v + 1];
    qsort(g->nb + a, (size_t)(b - a), sizeof(int32_t), cmp_i32);
    for (int32_t i = a; i < b; i++) {
      int32_t w = g->nb[i];
      if (w < 0 || w >= n || w == v) return ORC_ERR_NOT_SIMPLE;
      if (i > a && g->nb[i - 1] == w) return ORC_ERR_NOT_SIMPLE;
    }
  }
  for (int32_t v = 0; v < n; v++)
    for (int32_t i = g->start[v]; i < g->start[v + 1]; i++)
      if (!adjacent(g, g->nb[i], v)) return ORC_ERR_NOT_SIMPLE;
  return ORC_OK;
}

static void free_graph(orc_graph *g) {
  free(g->start);
  free(g->nb);
  memset(g, 0, sizeof(*g));
}

/* ------------------------------------------------------- degree labelling */
/* Section 2: G_1 = G, G_{i+1} = G_i - u_i with u_i of minimum degree in
 * G_i, l(u_i) = i.  Ties: smallest vertex id. */
static void degree_labelling(const orc_graph *g, int32_t *label) {
  int32_t n = g->n;
  int32_t *deg = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  char *alive = (char *)malloc((size_t)(n > 0 ? n : 1));
  for (int32_t v = 0; v < n; v++) {
    deg[v] = g->start[v + 1] - g->start[v];
    alive[v] = 1;
  }
  for (int32_t i = 0; i < n; i++) {
    int32_t u = -1;
    for (int32_t v = 0; v < n; v++)
      if (alive[v] && (u < 0 || deg[v] < deg[u])) u = v;
    label[u] = i;
    alive[u] = 0;
    for (int32_t k = g->start[u]; k < g->start[u + 1]; k++)
      if (alive[g->nb[k]]) deg[g->nb[k]]--;
  }
  free(deg);
  free(alive);
}

/* ------------------------------------------------------------ enumeration */
typedef struct {
  const orc_graph *g;
  const int32_t *label;
  int64_t *hist;   /* n+1 */
  int64_t *front;  /* n+1 */
  int32_t *path;   /* current path, original ids */
  int32_t *verts;  /* optional cycle sink */
  int64_t verts_cap, nverts;
  int64_t *offs;   /* cycle i occupies verts[offs[i] .. offs[i+1]) */
  int64_t cyc_cap, ncyc;
  int stored_all;  /* cleared at the first cycle that does not fit */
  int64_t repeat_violations;
} orc_run;

static void emit_cycle(orc_run *r, const int32_t *vs, int32_t k) {
  r->hist[k]++;
  if (r->stored_all && r->verts && r->offs && r->ncyc < r->cyc_cap &&
      r->nverts + k <= r->verts_cap) {
    memcpy(r->verts + r->nverts, vs, sizeof(int32_t) * (size_t)k);
    r->offs[r->ncyc] = r->nverts;
    r->offs[r->ncyc + 1] = r->nverts + k;
  } else {
    r->stored_all = 0;
  }
  r->ncyc++;
  r->nverts += k;
}

/* Algorithm 1, loop body, for the path r->path[0..t-1] (t >= 3). */
static void visit(orc_run *r, int32_t t) {
  const orc_graph *g = r->g;
  const int32_t *p = r->path;
  r->front[t]++;
  int32_t vt = p[t - 1];
  int32_t l2 = r->label[p[1]];
  for (int32_t k = g->start[vt]; k < g->start[vt + 1]; k++) {
    int32_t v = g->nb[k];
    if (r->label[v] <= l2) continue;                   /* l(v) > l(v2) */
    int chord = 0;
    for (int32_t i = 1; i <= t - 2 && !chord; i++)     /* v2 .. v(t-1) */
      chord = adjacent(g, v, p[i]);
    if (chord) continue;
    for (int32_t i = 0; i < t; i++)                    /* implied: v not on p */
      if (p[i] == v) r->repeat_violations++;
    r->path[t] = v;
    if (adjacent(g, v, p[0]))
      emit_cycle(r, r->path, t + 1);                   /* <p, v> is a cycle */
    else
      visit(r, t + 1);                                 /* <p, v> is a path  */
  }
}

/* Stage one visits the (u, x, y) choices with l(u) < l(x) < l(y) in a fixed
 * order (u by id, then x and y in sorted adjacency order); `root_lo` and
 * `root_hi` select a contiguous range of them so that a long run can be
 * split across processes.  Pass 0 and INT64_MAX for the whole graph. */
static void run_roots(orc_run *r, int64_t root_lo, int64_t root_hi) {
  const orc_graph *g = r->g;
  const int32_t *l = r->label;
  int64_t idx = 0;
  for (int32_t u = 0; u < g->n; u++)
    for (int32_t a = g->start[u]; a < g->start[u + 1]; a++)
      for (int32_t b = g->start[u]; b < g->start[u + 1]; b++) {
        int32_t x = g->nb[a], y = g->nb[b];
        if (!(l[u] < l[x] && l[x] < l[y])) continue;
        int64_t my = idx++;
        if (my < root_lo || my >= root_hi) continue;
        r->path[0] = x;
        r->path[1] = u;
        r->path[2] = y;
        if (adjacent(g, x, y))
          emit_cycle(r, r->path, 3);   /* triangle, into C directly */
        else
          visit(r, 3);                 /* initial triplet of T(G)   */
      }
}

/* ------------------------------------------------------------------- API */
int orc_validate(int32_t n, const int32_t *row_ptr, const int32_t *col_idx) {
  orc_graph g;
  int st = load_graph(n, row_ptr, col_idx, &g);
  free_graph(&g);
  return st;
}

int orc_degree_labelling(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                         int32_t *label_out) {
  orc_graph g;
  int st = load_graph(n, row_ptr, col_idx, &g);
  if (st == ORC_OK && n > 0) {
    if (!label_out) st = ORC_ERR_INVALID_ARG;
    else degree_labelling(&g, label_out);
  }
  free_graph(&g);
  return st;
}

/* Number of stage-one roots (triangles plus initial triplets). */
int64_t orc_count_roots(int32_t n, const int32_t *row_ptr, const int32_t *col_idx) {
  orc_graph g;
  int st = load_graph(n, row_ptr, col_idx, &g);
  if (st != ORC_OK) { free_graph(&g); return st; }
  int32_t *label = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  degree_labelling(&g, label);
  int64_t c = 0;
  for (int32_t u = 0; u < n; u++)
    for (int32_t a = g.start[u]; a < g.start[u + 1]; a++)
      for (int32_t b = g.start[u]; b < g.start[u + 1]; b++)
        if (label[u] < label[g.nb[a]] && label[g.nb[a]] < label[g.nb[b]]) c++;
  free(label);
  free_graph(&g);
  return c;
}

/*
 * Enumerates the chordless cycles reached from stage-one roots
 * [root_lo, root_hi).  hist and front must hold n+1 entries (zeroed here).
 * label_out (n entries) is optional.  If verts/offs are given, the cycles
 * are stored in path order as a CSR (offs needs cyc_cap+1 entries) as long
 * as they fit; n_cycles / n_verts always receive the full totals.
 * Returns ORC_OK, a validation error, or ORC_ERR_INTERNAL if a path vertex
 * was ever offered as an extension (which the path-extension property of
 * Section 2 rules out).
 */
int orc_enumerate(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                  int64_t root_lo, int64_t root_hi,
                  int64_t *hist, int64_t *front, int32_t *label_out,
                  int32_t *verts, int64_t verts_cap, int64_t *offs, int64_t cyc_cap,
                  int64_t *n_cycles, int64_t *n_verts) {
  if (!hist || !front) return ORC_ERR_INVALID_ARG;
  orc_graph g;
  int st = load_graph(n, row_ptr, col_idx, &g);
  memset(hist, 0, sizeof(int64_t) * ((size_t)(n > 0 ? n : 0) + 1));
  memset(front, 0, sizeof(int64_t) * ((size_t)(n > 0 ? n : 0) + 1));
  if (n_cycles) *n_cycles = 0;
  if (n_verts) *n_verts = 0;
  if (st != ORC_OK) { free_graph(&g); return st; }
  if (n == 0) { free_graph(&g); return ORC_OK; }
  int32_t *label = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  int32_t *path = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
  degree_labelling(&g, label);
  if (label_out) memcpy(label_out, label, sizeof(int32_t) * (size_t)n);
  orc_run r;
  memset(&r, 0, sizeof(r));
  r.g = &g;
  r.label = label;
  r.hist = hist;
  r.front = front;
  r.path = path;
  r.verts = verts;
  r.verts_cap = verts ? verts_cap : 0;
  r.offs = offs;
  r.cyc_cap = offs ? cyc_cap : 0;
  r.stored_all = 1;
  if (offs && cyc_cap >= 0) offs[0] = 0;
  run_roots(&r, root_lo, root_hi);
  if (n_cycles) *n_cycles = r.ncyc;
  if (n_verts) *n_verts = r.nverts;
  int rc = r.repeat_violations ? ORC_ERR_INTERNAL : ORC_OK;
  free(label);
  free(path);
  free_graph(&g);
  return rc;
}
