"""Batched enumeration (many graphs per call) against the CPU oracle, graph
by graph: persistent work-stealing launch and per-graph launches."""
import json
import os

import numpy as np
import pytest

import oracle
from paper_1410_4876_amd import graphgen as gg

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def cc():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a gfx950 device"
    from paper_1410_4876_amd import cc as mod
    mod.lib()
    return mod


def mixed_graphs(seed, count=60):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        kind = i % 6
        if kind == 0:
            n = int(rng.integers(3, 40))
            out.append(gg.er_gnm(n, min(int(n * rng.uniform(1.0, 2.2)), n * (n - 1) // 2), rng))
        elif kind == 1:
            out.append(gg.permute_random(gg.grid(int(rng.integers(2, 6)), int(rng.integers(2, 7))), rng))
        elif kind == 2:
            out.append(gg.wheel(int(rng.integers(4, 20))))
        elif kind == 3:
            out.append(gg.random_tree(int(rng.integers(1, 30)), rng))
        elif kind == 4:
            out.append(gg.complete_bipartite(int(rng.integers(1, 6)), int(rng.integers(1, 6))))
        else:
            out.append(gg.csr_from_edges(int(rng.integers(0, 4)), []))
    return out


def oracle_hists(graphs, width):
    h = np.zeros((len(graphs), width), np.int64)
    for i, g in enumerate(graphs):
        r = oracle.enumerate_cycles(g.n, g.row_ptr, g.col_idx, want_cycles=False)
        h[i, :r.hist.size] = r.hist
    return h


@pytest.mark.parametrize("seed", [1, 2])
def test_mixed_batch_both_modes(cc, seed):
    graphs = mixed_graphs(seed)
    b = gg.pack_batch(graphs)
    with cc.prepare_batch(b) as h:
        want = oracle_hists(graphs, h.max_n + 1)
        assert np.array_equal(h.histograms(), want)
        assert np.array_equal(h.histograms(per_graph_launch=True), want)
        lab = h.labels()
        for i, g in enumerate(graphs):
            o = b.graph_vtx_off
            assert np.array_equal(lab[o[i]:o[i + 1]], oracle.degree_labelling(g.n, g.row_ptr, g.col_idx))


def test_batch_two_word_graphs(cc):
    rng = np.random.default_rng(9)
    graphs = [gg.er_gnm(100, 125, rng), gg.cycle(128), gg.grid(4, 17), gg.wheel(70),
              gg.er_gnm(30, 70, rng)]
    b = gg.pack_batch(graphs)
    with cc.prepare_batch(b) as h:
        want = oracle_hists(graphs, h.max_n + 1)
        assert np.array_equal(h.histograms(), want)


def four_word_graphs(seed):
    """Graphs of 129 to 256 vertices (four-word bitsets) among small ones."""
    rng = np.random.default_rng(seed)
    return [gg.cycle(256),
            gg.permute_random(gg.disjoint_union(gg.grid(6, 8), gg.grid(5, 7), gg.cycle(100)), rng),
            gg.er_gnm(30, 60, rng),
            gg.wheel(150),
            gg.permute_random(gg.disjoint_union(gg.grid(5, 6), gg.grid(6, 6), gg.grid(4, 10),
                                                gg.grid(3, 10)), rng),
            gg.grid(3, 5),
            gg.cone(gg.cycle(150)),
            gg.cycle(129),
            gg.permute_random(gg.er_gnm(60, 100, rng), rng)]


def test_batch_four_word_graphs(cc):
    graphs = four_word_graphs(31)
    assert max(g.n for g in graphs) == cc.CC_MAX_BATCH_VERTICES
    b = gg.pack_batch(graphs)
    with cc.prepare_batch(b) as h:
        assert h.max_n == 256
        want = oracle_hists(graphs, h.max_n + 1)
        assert np.array_equal(h.histograms(), want)
        assert np.array_equal(h.histograms(per_graph_launch=True), want)
        lab = h.labels()
        for i, g in enumerate(graphs):
            o = b.graph_vtx_off
            assert np.array_equal(lab[o[i]:o[i + 1]], oracle.degree_labelling(g.n, g.row_ptr, g.col_idx))


def test_batch_rejects_graph_over_limit(cc):
    graphs = [gg.cycle(5), gg.cycle(cc.CC_MAX_BATCH_VERTICES + 1)]
    b = gg.pack_batch(graphs)
    with pytest.raises(cc.CCError) as ei:
        cc.Batch(b.graph_vtx_off, b.row_ptr, b.col_idx)
    assert ei.value.status == cc.CC_ERR_TOO_LARGE


def test_batch_repeated_and_tuned(cc):
    graphs = gg.er_batch_graphs(200, k=77)
    b = gg.pack_batch(graphs)
    want = None
    for wpc, dmin in [(0, 0), (4, 2), (32, 1 << 30)]:
        with cc.prepare_batch(b, dfs_waves_per_cu=wpc, dfs_donate_min=dmin) as h:
            if want is None:
                want = oracle_hists(graphs, h.max_n + 1)
            for _ in range(2):
                assert np.array_equal(h.histograms(), want)


def test_batch_rejects_bad_graph(cc):
    graphs = [gg.cycle(5), gg.cycle(6)]
    b = gg.pack_batch(graphs)
    ci = b.col_idx.copy()
    ci[0] = ci[1]  # duplicate neighbour in graph 0
    with pytest.raises(cc.CCError) as ei:
        cc.Batch(b.graph_vtx_off, b.row_ptr, ci)
    assert ei.value.status == cc.CC_ERR_NOT_SIMPLE


@pytest.mark.skipif(not os.path.exists(os.path.join(GOLDEN, "batch4096.json")),
                    reason="stored oracle output for the 4096-graph batch not generated")
def test_workload_batch4096(cc):
    """4096 ER graphs (n in [16, 64], d in [2.5, 5]) against the stored
    oracle histograms, persistent launch."""
    gold = json.load(open(os.path.join(GOLDEN, "batch4096.json")))
    b = gg.workload_batch4096()
    with cc.prepare_batch(b) as h:
        got = h.histograms()
        info = h.last_run()
    for i, want in enumerate(gold["hists"]):
        assert got[i, :len(want)].tolist() == want, f"graph {i}"
    assert info["paths"] == gold["total_paths"]


def test_batch_hist_off_places_each_graph(cc):
    """cc_histogram_batch's hist_off contract: graph g's n_g + 1 entries go to
    hists[hist_off[g]:], in any order and with gaps; nothing else is
    written.  Both launch forms."""
    graphs = mixed_graphs(5, count=24)
    b = gg.pack_batch(graphs)
    sizes = np.diff(b.graph_vtx_off)
    rng = np.random.default_rng(3)
    order = rng.permutation(len(graphs))
    off = np.zeros(len(graphs), np.int64)
    pos = 7
    for g in order:
        off[g] = pos
        pos += int(sizes[g]) + 1 + int(rng.integers(0, 4))
    with cc.prepare_batch(b) as h:
        want = oracle_hists(graphs, h.max_n + 1)
        for per_graph in (False, True):
            buf = np.full(pos + 5, -123, np.int64)
            h.histograms_into(buf, off, per_graph_launch=per_graph)
            touched = np.zeros(buf.size, bool)
            for g in range(len(graphs)):
                n_g = int(sizes[g])
                assert buf[off[g]:off[g] + n_g + 1].tolist() == want[g, :n_g + 1].tolist()
                touched[off[g]:off[g] + n_g + 1] = True
            assert (buf[~touched] == -123).all()
