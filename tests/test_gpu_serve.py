"""Serving loop (cc_server_*): requests submitted while others are on the
device come back with the same histogram as the graph run alone, and as the
CPU oracle; invalid, oversize and empty requests are answered without
disturbing the rest; small capacities split the stream into many batches
and no reply is lost or duplicated."""
import time

import numpy as np
import pytest

import oracle
from paper_1410_4876_amd import graphgen as gg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cc():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a gfx950 device"
    from paper_1410_4876_amd import cc as mod
    mod.lib()
    return mod


def alone(cc, g):
    with cc.prepare(g) as h:
        return h.histogram()


def oracle_hist(g):
    return oracle.enumerate_cycles(g.n, g.row_ptr, g.col_idx, want_cycles=False).hist


def small_stream(count, k):
    """Request-shaped graphs kept small enough for the oracle."""
    rng = np.random.default_rng(k)
    out = []
    for i in range(count):
        if i % 2 == 0:
            out.append(gg.permute_random(gg.grid(int(rng.integers(3, 6)), int(rng.integers(3, 6))), rng))
        else:
            n = int(rng.integers(20, 50))
            out.append(gg.permute_random(gg.er_gnm(n, int(n * rng.uniform(1.2, 1.8)), rng), rng))
    return out


def test_stream_matches_alone_and_oracle(cc):
    reqs = gg.request_stream(max_requests=160, k=5)
    graphs = [r.graph for r in reqs]
    with cc.Server() as sv:
        ids = []
        t0 = time.perf_counter()
        for r in reqs:  # submit on the stream's own clock, so batches overlap
            delay = r.arrival_s - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
            ids.append(sv.submit_graph(r.graph))
        got = [sv.result(i, timeout_s=120.0) for i in ids]
        st = sv.stats()
    assert st["completed"] == len(reqs) and st["pending"] == 0
    for g, (h, lat, status) in zip(graphs, got):
        assert status == cc.CC_OK
        assert lat >= 0.0
        assert np.array_equal(h, alone(cc, g))
    for g, (h, _, _) in list(zip(graphs, got))[:12]:
        if g.n <= 40:
            want = oracle_hist(g)
            assert np.array_equal(h[:want.size], want)


def test_small_capacities_many_batches(cc):
    graphs = small_stream(90, 11)
    with cc.Server(slots=2, max_batch_graphs=3) as sv:
        ids = [sv.submit_graph(g) for g in graphs]
        got = [sv.result(i, timeout_s=120.0) for i in ids]
        st = sv.stats()
    assert st["batches"] >= 30 and st["max_batch"] <= 3 and st["completed"] == 90
    for g, (h, _, status) in zip(graphs, got):
        assert status == cc.CC_OK
        want = oracle_hist(g)
        assert np.array_equal(h[:want.size], want) and not h[want.size:].any()


def test_invalid_empty_and_oversize_requests(cc):
    good = small_stream(20, 12)
    loop = gg.csr_from_edges(4, [(0, 1), (1, 2), (2, 3), (3, 0)])
    self_loop_rp = np.array([0, 2, 3, 4], np.int32)
    self_loop_ci = np.array([1, 0, 0, 0], np.int32)   # vertex 0 lists itself
    out_of_range_ci = np.array([1, 7, 0, 0], np.int32)
    asym_rp = np.array([0, 1, 1, 1], np.int32)
    asym_ci = np.array([1], np.int32)
    big = gg.complete(40)  # 40 * C(39, 2) root slots
    with cc.Server(slots=2, slot_root_slots=20000) as sv:
        ids = []
        for i, g in enumerate(good):
            ids.append(("good", g, sv.submit_graph(g)))
            if i == 5:
                ids.append(("bad", None, sv.submit(3, self_loop_rp, self_loop_ci)))
                ids.append(("bad", None, sv.submit(3, self_loop_rp, out_of_range_ci)))
                ids.append(("bad", None, sv.submit(3, asym_rp, asym_ci)))
            if i == 9:
                ids.append(("empty", gg.csr_from_edges(0, []), sv.submit(0, [0], [])))
                ids.append(("empty", gg.csr_from_edges(1, []), sv.submit(1, [0, 0], [])))
                ids.append(("big", big, sv.submit_graph(big)))
                ids.append(("good", loop, sv.submit_graph(loop)))
        for kind, g, rid in ids:
            h, _, status = sv.result(rid, timeout_s=120.0)
            if kind == "bad":
                assert status == cc.CC_ERR_NOT_SIMPLE
            elif kind == "big":
                assert status == cc.CC_ERR_OUT_OF_MEMORY
            else:
                assert status == cc.CC_OK
                want = oracle_hist(g)
                assert np.array_equal(h[:want.size], want)
        assert sv.stats()["rejected"] == 1


def test_result_timeout_keeps_the_request(cc):
    g = gg.grid(6, 6)
    with cc.Server() as sv:
        rid = sv.submit_graph(g)
        try:
            h, _, status = sv.result(rid, timeout_s=0.0)
        except cc.CCError as e:
            assert e.status == cc.CC_ERR_NOT_READY
            h, _, status = sv.result(rid, timeout_s=120.0)
        assert status == cc.CC_OK
        assert np.array_equal(h, alone(cc, g))


def test_four_word_requests(cc):
    rng = np.random.default_rng(22)
    graphs = [gg.cycle(256), gg.wheel(150), gg.cone(gg.cycle(140)),
              gg.permute_random(gg.disjoint_union(gg.grid(6, 8), gg.grid(5, 7), gg.cycle(100)), rng)]
    graphs += small_stream(10, 14)
    with cc.Server() as sv:
        with pytest.raises(cc.CCError) as ei:
            sv.submit_graph(gg.cycle(cc.CC_MAX_BATCH_VERTICES + 1))
        assert ei.value.status == cc.CC_ERR_TOO_LARGE
        ids = [sv.submit_graph(g) for g in graphs]
        for g, rid in zip(graphs, ids):
            h, _, status = sv.result(rid, timeout_s=120.0)
            assert status == cc.CC_OK
            assert np.array_equal(h, alone(cc, g))


def test_two_word_requests(cc):
    rng = np.random.default_rng(21)
    graphs = [gg.permute_random(gg.er_gnm(n, int(n * 1.25), rng), rng) for n in (70, 90, 100, 128)]
    graphs += small_stream(10, 13)
    with cc.Server() as sv:
        ids = [sv.submit_graph(g) for g in graphs]
        for g, rid in zip(graphs, ids):
            h, _, status = sv.result(rid, timeout_s=120.0)
            assert status == cc.CC_OK
            assert np.array_equal(h, alone(cc, g))
