"""Graphs of 257 to 1024 vertices (eight- and sixteen-word bitsets, rows
read from device memory, 16-bit end vertices) against the oracle: every
cycle, the histogram, the labels and the expanded-path counts, through the
breadth-first steps, a forced or budget-driven depth-first hand-over, and
the sorted output (vertex ids above 255: two byte digits per position)."""
import numpy as np
import pytest

import oracle
from ccutil import canonical_groups
from paper_1410_4876_amd import graphgen as gg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cc():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a gfx950 device"
    from paper_1410_4876_amd import cc as mod
    mod.lib()
    return mod


def rng(seed):
    return np.random.default_rng(seed)


def union774():
    """774 vertices, ids permuted: four 6x8 and four 5x7 grids, C_300, a
    100-spoke wheel, K_{4,5} and the 5-cube (231870 chordless cycles of 3 to
    300 vertices)."""
    parts = [gg.grid(6, 8)] * 4 + [gg.grid(5, 7)] * 4 + [
        gg.cycle(300), gg.wheel(100), gg.complete_bipartite(4, 5), gg.hypercube(5)]
    return gg.permute_random(gg.disjoint_union(*parts), rng(774))


def big_suite():
    return [
        gg.cycle(257), gg.cycle(300), gg.cycle(512), gg.cycle(513), gg.cycle(1024),
        gg.wheel(600),  # a hub of degree 600
        gg.permute_random(gg.cone(gg.cycle(1000)), rng(1001)),
        gg.tree_plus_edges(400, 18, rng(2)),
        gg.tree_plus_edges(1000, 14, rng(1)),
        gg.permute_random(gg.tree_plus_edges(1024, 20, rng(3)), rng(33)),
        union774(),
    ]


def oracle_run(g, cycles=True):
    return oracle.enumerate_cycles(g.n, g.row_ptr, g.col_idx, want_cycles=cycles)


def check(cc, g, **kw):
    import torch
    ores = oracle_run(g)
    with cc.prepare(g, **kw) as h:
        verts, offs = h.enumerate()
        torch.cuda.synchronize()
        v, o = verts.cpu().numpy(), offs.cpu().numpy()
        assert np.array_equal(h.histogram(), ores.hist)
        assert np.array_equal(h.labels(), ores.labels)
        assert np.array_equal(h.frontier(), ores.front)
        info = h.last_run()
        assert h.count() == ores.count
    assert np.all(np.diff(np.diff(o)) >= 0), "output not ordered by length"
    a, b = canonical_groups(v, o), canonical_groups(*ores.cycles)
    assert sorted(a) == sorted(b)
    for k in a:
        assert np.array_equal(a[k], b[k]), f"cycles of length {k} differ"
    return info


@pytest.mark.parametrize("g", big_suite(), ids=lambda g: f"{g.name[:24]}_n{g.n}_m{g.m}")
def test_big_graph_parity(cc, g):
    check(cc, g)


@pytest.mark.parametrize("case,level", [("c1024", 3), ("tree1024", 3), ("tree1024", 9),
                                        ("union774", 4), ("union774", 40), ("wheel600", 3),
                                        ("c512", 3), ("c512", 100), ("tree400", 4)])
def test_big_graph_forced_depth_first(cc, case, level):
    g = {"c1024": lambda: gg.cycle(1024), "c512": lambda: gg.cycle(512),
         "tree1024": lambda: gg.permute_random(gg.tree_plus_edges(1024, 20, rng(3)), rng(33)),
         "tree400": lambda: gg.permute_random(gg.tree_plus_edges(400, 18, rng(2)), rng(22)),
         "union774": union774, "wheel600": lambda: gg.wheel(600)}[case]()
    info = check(cc, g, force_dfs_level=level)
    assert info["switch_level"] == level


@pytest.mark.parametrize("budget", [1 << 20, 8 << 20])
def test_big_graph_budget_switch(cc, budget):
    # 1 MiB holds about a thousand paths per level (enumerate mode, sixteen
    # words): the hand-over comes at once; 8 MiB holds levels up to 7
    # (5183 paths) but not level 8 (9103)
    info = check(cc, union774(), budget_bytes=budget)
    assert info["switch_level"] >= 3
    if budget > 1 << 20:
        assert info["switch_level"] > 3


@pytest.mark.parametrize("case,output_device", [("union774", True), ("union774", False),
                                                 ("tree400", True)])
def test_big_graph_sorted_output(cc, case, output_device):
    """CC_SORTED with original ids up to 773 (sixteen-word bitsets) and 399
    (eight words): exactly the oracle's sorted canonical list."""
    import torch
    g = union774() if case == "union774" else gg.permute_random(
        gg.tree_plus_edges(400, 18, rng(2)), rng(22))
    with cc.prepare(g, sorted_output=True, output_device=output_device,
                    force_dfs_level=6) as h:
        v, o = h.enumerate()
        if output_device:
            torch.cuda.synchronize()
            v, o = v.cpu().numpy(), o.cpu().numpy()
    groups = canonical_groups(*oracle_run(g).cycles)
    want_v = np.concatenate([groups[k].reshape(-1) for k in sorted(groups)])
    want_o = np.concatenate([[0], np.cumsum([k for k in sorted(groups)
                                             for _ in range(groups[k].shape[0])])])
    assert np.array_equal(np.asarray(o, np.int64), want_o)
    assert np.array_equal(np.asarray(v, np.int64)[:want_v.size], want_v)


def test_big_graph_root_ranges_and_grouping(cc):
    """Stage-one root ranges and the root-grouped output on a 1024-vertex
    graph: each range equals the oracle's run over it."""
    import torch
    g = gg.permute_random(gg.tree_plus_edges(1024, 20, rng(3)), rng(33))
    ores = oracle_run(g)
    nc, nv = int(ores.hist.sum()), int((ores.hist * np.arange(g.n + 1)).sum())
    total = oracle.count_roots(g.n, g.row_ptr, g.col_idx)
    cuts = sorted(set([0, total] + [int(x) for x in rng(5).integers(0, total + 1, 3)]))
    with cc.prepare(g) as h:
        assert h.root_total() == total
        v = torch.empty(max(nv, 1), dtype=torch.int32, device="cuda")
        o = torch.empty(nc + 1, dtype=torch.int64, device="cuda")
        f = torch.empty(total + 1, dtype=torch.int64, device="cuda")
        assert h.enumerate_by_roots_into(v, o, f) == (nc, nv)
        torch.cuda.synchronize()
        v, o, f = v.cpu().numpy(), o.cpu().numpy(), f.cpu().numpy()
        for lo, hi in zip(cuts[:-1], cuts[1:]):
            rres = oracle.enumerate_cycles(g.n, g.row_ptr, g.col_idx, want_cycles=True,
                                           root_lo=lo, root_hi=hi)
            assert np.array_equal(h.histogram_roots(lo, hi), rres.hist), (lo, hi)
            c0, c1 = int(f[lo]), int(f[hi])
            a = canonical_groups(v[o[c0]:o[c1]], o[c0:c1 + 1] - o[c0])
            b = canonical_groups(*rres.cycles)
            assert sorted(a) == sorted(b) and all(np.array_equal(a[k], b[k]) for k in a)
    assert f[0] == 0 and f[-1] == nc and o[-1] == nv
