"""Test-side helpers: canonical cycle form, an independent brute-force
enumerator, and small graph utilities.  Neither the oracle nor the HIP path
imports this module."""
from __future__ import annotations

import numpy as np


def adjacency_sets(n, row_ptr, col_idx):
    return [set(int(w) for w in col_idx[row_ptr[v]:row_ptr[v + 1]]) for v in range(n)]


def canonical(cycle) -> tuple:
    """Rotate a cycle (vertex sequence, first vertex not repeated) so that it
    starts at its minimum vertex id and continues towards the smaller of that
    vertex's two cycle neighbours."""
    c = [int(x) for x in cycle]
    k = len(c)
    i = c.index(min(c))
    fwd, bwd = c[(i + 1) % k], c[(i - 1) % k]
    if fwd <= bwd:
        return tuple(c[(i + j) % k] for j in range(k))
    return tuple(c[(i - j) % k] for j in range(k))


def canonical_sorted(cycles) -> list:
    return sorted((canonical(c) for c in cycles), key=lambda t: (len(t), t))


def is_chordless_cycle(cycle, adj) -> bool:
    """Checks the definition directly: consecutive vertices adjacent
    (cyclically), all distinct, and no other pair adjacent."""
    c = [int(x) for x in cycle]
    k = len(c)
    if k < 3 or len(set(c)) != k:
        return False
    for i in range(k):
        for j in range(i + 1, k):
            consecutive = (j == i + 1) or (i == 0 and j == k - 1)
            if (c[j] in adj[c[i]]) != consecutive:
                return False
    return True


def brute_force_sets(n, row_ptr, col_idx):
    """All vertex sets S (|S| >= 3) whose induced subgraph is connected and
    2-regular, i.e. all chordless cycles as frozensets.  Exhaustive over the
    2^n subsets; intended for n <= 16."""
    assert n <= 20
    adj = np.zeros(n, dtype=np.uint32)
    for v in range(n):
        for w in col_idx[row_ptr[v]:row_ptr[v + 1]]:
            adj[v] |= np.uint32(1) << np.uint32(w)
    if n == 0:
        return []
    S = np.arange(1 << n, dtype=np.uint32)
    ok = np.bitwise_count(S) >= 3
    for v in range(n):
        inS = (S >> np.uint32(v)) & np.uint32(1)
        d = np.bitwise_count(S & adj[v])
        ok &= (inS == 0) | (d == 2)
    out = []
    for s in np.nonzero(ok)[0]:
        s = int(s)
        # connectivity of G[S] by flood fill
        start = (s & -s).bit_length() - 1
        seen = 1 << start
        frontier = seen
        while frontier:
            nxt = 0
            f = frontier
            while f:
                v = (f & -f).bit_length() - 1
                f &= f - 1
                nxt |= int(adj[v]) & s
            nxt &= ~seen
            seen |= nxt
            frontier = nxt
        if seen == s:
            out.append(frozenset(v for v in range(n) if s >> v & 1))
    return out


def hist_of_sets(sets, n):
    h = np.zeros(n + 1, np.int64)
    for s in sets:
        h[len(s)] += 1
    return h


def dense_adjacency(n, row_ptr, col_idx):
    A = np.zeros((n, n), dtype=np.int64)
    for v in range(n):
        A[v, col_idx[row_ptr[v]:row_ptr[v + 1]]] = 1
    return A


def triangles_by_trace(n, row_ptr, col_idx) -> int:
    A = dense_adjacency(n, row_ptr, col_idx)
    return int(np.trace(A @ A @ A) // 6)


def canonical_groups(verts, offs):
    """Canonicalise a CSR of cycles (any rotation/direction) and group by
    length: returns {k: (N_k, k) int64 array, rows sorted lexicographically}.
    Vectorised per length."""
    verts = np.asarray(verts, dtype=np.int64)
    offs = np.asarray(offs, dtype=np.int64)
    lens = np.diff(offs)
    out = {}
    for k in np.unique(lens):
        k = int(k)
        starts = offs[:-1][lens == k]
        a = verts[starts[:, None] + np.arange(k)[None, :]]
        i = np.argmin(a, axis=1)
        fwd = a[np.arange(a.shape[0]), (i + 1) % k]
        bwd = a[np.arange(a.shape[0]), (i - 1) % k]
        step = np.where(fwd <= bwd, 1, -1)
        idx = (i[:, None] + step[:, None] * np.arange(k)[None, :]) % k
        c = np.take_along_axis(a, idx, axis=1)
        order = np.lexsort(c.T[::-1])
        out[k] = c[order]
    return out


def is_canonical_array(verts, offs) -> bool:
    """True if every cycle already starts at its minimum and continues towards
    the smaller neighbour."""
    verts = np.asarray(verts, dtype=np.int64)
    offs = np.asarray(offs, dtype=np.int64)
    lens = np.diff(offs)
    for k in np.unique(lens):
        k = int(k)
        starts = offs[:-1][lens == k]
        a = verts[starts[:, None] + np.arange(k)[None, :]]
        if not np.all(a[:, 0] == a.min(axis=1)):
            return False
        if k >= 3 and not np.all(a[:, 1] <= a[:, -1]):
            return False
    return True


def groups_digest(groups) -> str:
    """sha256 over the canonical sorted cycles, lengths ascending."""
    import hashlib
    h = hashlib.sha256()
    for k in sorted(groups):
        h.update(np.int64(k).tobytes())
        h.update(np.ascontiguousarray(groups[k], dtype=np.int64).tobytes())
    return h.hexdigest()


def groups_all_chordless(groups, n, row_ptr, col_idx) -> bool:
    """Every row of every group (k vertex ids) is a chordless cycle in the
    vertex order given: k distinct vertices, consecutive ones adjacent
    (cyclically), and exactly k edges among them (so no chord).  Vectorised
    over the rows with per-vertex adjacency bitsets."""
    words = max(1, (n + 63) // 64)
    adj = np.zeros((max(n, 1), words), dtype=np.uint64)
    for v in range(n):
        for w in col_idx[row_ptr[v]:row_ptr[v + 1]]:
            adj[v, int(w) // 64] |= np.uint64(1) << np.uint64(int(w) % 64)
    one = np.uint64(1)
    for k, a in groups.items():
        a = np.asarray(a, dtype=np.int64)
        if a.shape[0] == 0:
            continue
        S = np.zeros((a.shape[0], words), dtype=np.uint64)
        for i in range(k):
            for w in range(words):
                sel = (a[:, i] // 64) == w
                S[sel, w] |= one << (a[sel, i] % 64).astype(np.uint64)
        if not np.all(np.bitwise_count(S).sum(axis=1) == k):
            return False  # repeated vertex
        deg2 = np.zeros(a.shape[0], dtype=np.int64)
        for i in range(k):
            deg2 += np.bitwise_count(adj[a[:, i]] & S).sum(axis=1).astype(np.int64)
            nxt = a[:, (i + 1) % k]
            bit = (adj[a[:, i], nxt // 64] >> (nxt % 64).astype(np.uint64)) & one
            if not np.all(bit == one):
                return False  # consecutive vertices not adjacent
        if not np.all(deg2 == 2 * k):
            return False  # a chord
    return True


def brute_force_front(n, row_ptr, col_idx, labels):
    """front[t] by brute force: the vertex sequences (v1, ..., vt), t >= 3,
    that form an induced path (distinct, consecutive ones adjacent, no other
    pair adjacent) whose second vertex has the smallest label of the path and
    whose first vertex has a smaller label than its third.  These are exactly
    the open chordless paths the method expands (Section 2): the initial
    triplets for t = 3 and their extensions.  Depth-first over sequences;
    intended for n <= 10."""
    adj = adjacency_sets(n, row_ptr, col_idx)
    lab = [int(x) for x in labels]
    front = np.zeros(n + 1, np.int64)

    def grow(path):
        t = len(path)
        if t >= 3:
            front[t] += 1
        last = path[-1]
        for v in adj[last]:
            if v in path or lab[v] < lab[path[1]]:
                continue
            if any(v in adj[u] for u in path[:-1]):
                continue  # a chord, or a closure through v1
            if t == 2 and lab[path[0]] > lab[v]:
                continue
            grow(path + [v])

    for v1 in range(n):
        for v2 in adj[v1]:
            if lab[v2] < lab[v1]:
                grow([v1, v2])
    return front
