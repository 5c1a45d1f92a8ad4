"""Seeded synthetic graph generators (inputs only).

This module builds undirected simple graphs as int32 CSR arrays.  It holds
none of the enumeration method's arithmetic: no labelling, no triplets, no
path expansion.  Both the CPU oracle and the HIP path read graphs made here,
so parity is always checked on byte-identical inputs.

CSR convention used everywhere in this project: ``row_ptr`` has n+1 int32
entries, ``col_idx`` has 2m int32 entries, each undirected edge {a, b}
appears once in a's list and once in b's, and every list is sorted.

Workload shapes follow the paper's experimental graphs (Section 5, Table 1:
grids, cycles, wheels, complete bipartite graphs) plus sparse Erdos-Renyi
G(n, m) graphs of comparable size.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass

import numpy as np

SEED_BASE = 14104876


def rng_for(k: int) -> np.random.Generator:
    """Generator for workload k (seed = 14104876 + k)."""
    return np.random.default_rng(SEED_BASE + k)


# --------------------------------------------------------------------------
# CSR assembly
# --------------------------------------------------------------------------
@dataclass
class CSR:
    n: int
    row_ptr: np.ndarray  # int32 [n+1]
    col_idx: np.ndarray  # int32 [2m]
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.col_idx.shape[0] // 2)

    @property
    def max_degree(self) -> int:
        if self.n == 0:
            return 0
        return int(np.max(np.diff(self.row_ptr))) if self.n else 0

    def edges(self) -> np.ndarray:
        """Edge list [m, 2] with a < b."""
        src = np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.row_ptr))
        dst = self.col_idx.astype(np.int64)
        keep = src < dst
        return np.stack([src[keep], dst[keep]], axis=1)


def csr_from_edges(n: int, edges, name: str = "") -> CSR:
    """Build a sorted, symmetric CSR from an iterable of (a, b) pairs.

    Self-loops and duplicate edges are rejected: the generators only ever
    produce simple graphs.
    """
    e = np.asarray(list(edges) if not isinstance(edges, np.ndarray) else edges,
                   dtype=np.int64).reshape(-1, 2)
    if e.size:
        if np.any(e[:, 0] == e[:, 1]):
            raise ValueError("self-loop in generator output")
        lo = np.minimum(e[:, 0], e[:, 1])
        hi = np.maximum(e[:, 0], e[:, 1])
        if np.any(lo < 0) or np.any(hi >= n):
            raise ValueError("vertex id out of range")
        key = lo * max(n, 1) + hi
        if np.unique(key).size != key.size:
            raise ValueError("duplicate edge in generator output")
        src = np.concatenate([lo, hi])
        dst = np.concatenate([hi, lo])
    else:
        src = np.zeros(0, np.int64)
        dst = np.zeros(0, np.int64)
    order = np.lexsort((dst, src))
    src, dst = src[order], dst[order]
    counts = np.bincount(src, minlength=n) if n else np.zeros(0, np.int64)
    row_ptr = np.zeros(n + 1, dtype=np.int32)
    if n:
        row_ptr[1:] = np.cumsum(counts)
    return CSR(n, row_ptr, dst.astype(np.int32), name)


def permute(g: CSR, perm: np.ndarray, name: str | None = None) -> CSR:
    """Relabel vertex v as perm[v]."""
    perm = np.asarray(perm, dtype=np.int64)
    e = g.edges()
    return csr_from_edges(g.n, perm[e] if e.size else e, name or g.name)


def permute_random(g: CSR, rng: np.random.Generator) -> CSR:
    return permute(g, rng.permutation(g.n), g.name + "-perm")


# --------------------------------------------------------------------------
# Families
# --------------------------------------------------------------------------
def er_gnm(n: int, m: int, rng: np.random.Generator, name: str | None = None) -> CSR:
    """G(n, m): m distinct pairs drawn uniformly without replacement from the
    C(n, 2) unordered pairs, the pair index unranked lexicographically
    ((0,1), (0,2), ..., (0,n-1), (1,2), ...)."""
    total = n * (n - 1) // 2
    if m > total:
        raise ValueError("m exceeds C(n,2)")
    idx = np.sort(rng.choice(total, size=m, replace=False)) if m else np.zeros(0, np.int64)
    # Unrank: row a holds pairs (a, a+1..n-1); its first index is
    # a*n - a*(a+1)/2.
    starts = np.array([r * n - r * (r + 1) // 2 for r in range(max(n, 1))], dtype=np.int64)
    a = np.searchsorted(starts, idx, side="right") - 1
    b = idx - starts[a] + a + 1
    return csr_from_edges(n, np.stack([a, b], axis=1), name or f"er_{n}_{m}")


def grid(p: int, q: int, name: str | None = None) -> CSR:
    """p x q square grid; vertex (r, c) has id r*q + c."""
    e = []
    for r in range(p):
        for c in range(q):
            v = r * q + c
            if c + 1 < q:
                e.append((v, v + 1))
            if r + 1 < p:
                e.append((v, v + q))
    return csr_from_edges(p * q, e, name or f"grid_{p}x{q}")


def cycle(n: int) -> CSR:
    return csr_from_edges(n, [(i, (i + 1) % n) for i in range(n)], f"C{n}")


def path_graph(n: int) -> CSR:
    return csr_from_edges(n, [(i, i + 1) for i in range(n - 1)], f"P{n}")


def complete(n: int) -> CSR:
    return csr_from_edges(n, list(itertools.combinations(range(n), 2)), f"K{n}")


def complete_multipartite(*parts: int) -> CSR:
    owner = []
    for pi, s in enumerate(parts):
        owner += [pi] * s
    n = len(owner)
    e = [(a, b) for a, b in itertools.combinations(range(n), 2) if owner[a] != owner[b]]
    return csr_from_edges(n, e, "K" + "_".join(map(str, parts)))


def complete_bipartite(a: int, b: int) -> CSR:
    return complete_multipartite(a, b)


def wheel(rim: int) -> CSR:
    """Hub 0 joined to a rim cycle 1..rim (n = rim + 1 vertices)."""
    e = [(0, i) for i in range(1, rim + 1)]
    e += [(i, i % rim + 1) for i in range(1, rim + 1)]
    return csr_from_edges(rim + 1, e, f"wheel{rim}")


def ladder(q: int) -> CSR:
    return grid(2, q, f"ladder{q}")


def hypercube(d: int) -> CSR:
    n = 1 << d
    e = [(v, v ^ (1 << b)) for v in range(n) for b in range(d) if v < v ^ (1 << b)]
    return csr_from_edges(n, e, f"Q{d}")


def random_tree(n: int, rng: np.random.Generator) -> CSR:
    e = [(int(rng.integers(0, i)), i) for i in range(1, n)]
    return csr_from_edges(n, e, f"tree{n}")


def tree_plus_edges(n: int, extra: int, rng: np.random.Generator) -> CSR:
    """A random recursive tree on n vertices plus `extra` random non-tree
    edges: sparse, with few but long chordless cycles (at most 2^extra
    cycles in all, as the cycle space has dimension extra)."""
    e = {(int(rng.integers(0, i)), i) for i in range(1, n)}
    while len(e) < n - 1 + extra:
        a, b = (int(x) for x in rng.integers(0, n, 2))
        if a != b:
            e.add((min(a, b), max(a, b)))
    return csr_from_edges(n, sorted(e), f"tree{n}+{extra}")


def random_k_tree(n: int, k: int, rng: np.random.Generator) -> CSR:
    """A k-tree: start from K_{k+1}; each new vertex joins a random existing
    k-clique.  k-trees are chordal."""
    if n <= k:
        return complete(n)
    cliques = [tuple(range(k + 1))]
    e = set(itertools.combinations(range(k + 1), 2))
    kcl = [c for c in itertools.combinations(range(k + 1), k)]
    for v in range(k + 1, n):
        base = kcl[int(rng.integers(0, len(kcl)))]
        for w in base:
            e.add((w, v))
        for sub in itertools.combinations(base, k - 1):
            kcl.append(tuple(sorted(sub + (v,))))
        cliques.append(base + (v,))
    return csr_from_edges(n, sorted(e), f"{k}tree{n}")


def cone(g: CSR) -> CSR:
    """Add a universal vertex (id n) joined to every vertex of g."""
    e = [tuple(x) for x in g.edges()] + [(v, g.n) for v in range(g.n)]
    return csr_from_edges(g.n + 1, e, g.name + "+apex")


def disjoint_union(*gs: CSR) -> CSR:
    e, off = [], 0
    for g in gs:
        e += [(a + off, b + off) for a, b in g.edges()]
        off += g.n
    return csr_from_edges(off, e, "+".join(g.name for g in gs))


def from_adjacency_bits(n: int, bits: int) -> CSR:
    """Graph on n vertices whose edge set is the bitmask over the C(n, 2)
    pairs in lexicographic order (used for exhaustive small-n sweeps)."""
    e = [pr for i, pr in enumerate(itertools.combinations(range(n), 2)) if bits >> i & 1]
    return csr_from_edges(n, e, f"g{n}_{bits}")


# --------------------------------------------------------------------------
# Packed batches (disjoint union with per-graph vertex offsets)
# --------------------------------------------------------------------------
@dataclass
class Batch:
    graphs: list
    graph_vtx_off: np.ndarray  # int32 [G+1]
    row_ptr: np.ndarray        # int32 [N+1] over the union, global vertex ids
    col_idx: np.ndarray        # int32 [2M], global vertex ids


def pack_batch(graphs) -> Batch:
    """Pack graphs into one CSR; graph g owns vertices
    [graph_vtx_off[g], graph_vtx_off[g+1])."""
    offs = np.zeros(len(graphs) + 1, dtype=np.int64)
    for i, g in enumerate(graphs):
        offs[i + 1] = offs[i] + g.n
    N = int(offs[-1])
    rp = np.zeros(N + 1, dtype=np.int64)
    cols = []
    for i, g in enumerate(graphs):
        o = int(offs[i])
        rp[o + 1:o + g.n + 1] = g.row_ptr[1:].astype(np.int64)
        cols.append(g.col_idx.astype(np.int64) + o)
    # convert per-graph relative row pointers into global ones
    edge_base = 0
    for i, g in enumerate(graphs):
        o = int(offs[i])
        rp[o + 1:o + g.n + 1] += edge_base
        edge_base += int(g.col_idx.shape[0])
    col = np.concatenate(cols) if cols else np.zeros(0, np.int64)
    if N >= (1 << 31) or col.size >= (1 << 31):
        raise ValueError("batch too large for int32 CSR")
    return Batch(list(graphs), offs.astype(np.int32), rp.astype(np.int32), col.astype(np.int32))


# --------------------------------------------------------------------------
# Workloads (sizes from the project's five configurations)
# --------------------------------------------------------------------------
def workload_er40() -> CSR:
    """ER G(40, 100), seed index 1."""
    return er_gnm(40, 100, rng_for(1), "er_40_100")


def workload_grid8x8() -> CSR:
    """8x8 grid (n=64, m=112), ids permuted, seed index 2."""
    return permute_random(grid(8, 8), rng_for(2))


def workload_grid7x12() -> CSR:
    """7x12 grid (n=84, m=149), ids permuted, seed index 3.

    A p x q grid has 2pq - p - q edges; 7x12 therefore has 149 edges."""
    return permute_random(grid(7, 12), rng_for(3))


def er_batch_graphs(count: int, k: int, n_lo=16, n_hi=64, d_lo=2.5, d_hi=5.0):
    """`count` ER graphs: n ~ U{n_lo..n_hi}, d ~ U[d_lo, d_hi],
    m = floor(n*d/2 + 0.5) capped at C(n,2)."""
    rng = rng_for(k)
    out = []
    for i in range(count):
        n = int(rng.integers(n_lo, n_hi + 1))
        d = float(rng.uniform(d_lo, d_hi))
        m = min(int(np.floor(n * d / 2 + 0.5)), n * (n - 1) // 2)
        out.append(er_gnm(n, m, rng, f"er{i}_{n}_{m}"))
    return out


def workload_batch4096(count: int = 4096, k: int = 4) -> Batch:
    """4096 ER graphs, n in [16, 64], d in [2.5, 5], one packed CSR."""
    return pack_batch(er_batch_graphs(count, k))


@dataclass
class Request:
    arrival_s: float
    graph: CSR


def request_stream(rate_hz: float = 2000.0, duration_s: float = 60.0, k: int = 5,
                   max_requests: int | None = None):
    """Poisson request stream: exponential inter-arrival gaps at `rate_hz`.
    Each request is, with probability 1/2, a p x q grid (p, q ~ U{3..7}) or
    an ER graph (n ~ U{20..80}, d ~ U[3, 5]); ids permuted."""
    rng = rng_for(k)
    t = 0.0
    out = []
    while True:
        t += float(rng.exponential(1.0 / rate_hz))
        if t >= duration_s or (max_requests is not None and len(out) >= max_requests):
            break
        if rng.random() < 0.5:
            p = int(rng.integers(3, 8))
            q = int(rng.integers(3, 8))
            g = permute_random(grid(p, q), rng)
        else:
            n = int(rng.integers(20, 81))
            d = float(rng.uniform(3.0, 5.0))
            m = min(int(np.floor(n * d / 2 + 0.5)), n * (n - 1) // 2)
            g = permute_random(er_gnm(n, m, rng), rng)
        out.append(Request(t, g))
    return out
