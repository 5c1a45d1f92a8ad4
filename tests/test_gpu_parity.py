"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Results are exact: the sorted set of canonical cycles, the per-length
histogram, the degree labels and the per-length counts of expanded paths
must all be equal.  Large workloads compare against stored oracle outputs
(tests/golden, written by tests/golden/make_golden.py)."""
import json
import os

import numpy as np
import pytest

import oracle
from ccutil import canonical_groups, groups_digest, is_canonical_array
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


def oracle_run(g, cycles=True):
    return oracle.enumerate_cycles(g.n, g.row_ptr, g.col_idx, want_cycles=cycles)


def gpu_enumerate(cc, g, **kw):
    import torch
    with cc.prepare(g, **kw) as h:
        verts, offs = h.enumerate()
        torch.cuda.synchronize()
        return (verts.cpu().numpy(), offs.cpu().numpy(), h.histogram(), h.labels(),
                h.frontier(), h.last_run())


def assert_same_cycles(gpu_verts, gpu_offs, ores, by_length=True):
    assert is_canonical_array(gpu_verts, gpu_offs)
    if by_length:
        assert np.all(np.diff(np.diff(gpu_offs)) >= 0), "output not ordered by length"
    a = canonical_groups(gpu_verts, gpu_offs)
    b = canonical_groups(*ores.cycles)
    assert sorted(a) == sorted(b)
    for k in a:
        assert np.array_equal(a[k], b[k]), f"cycles of length {k} differ"
        if a[k].shape[0] > 1:
            assert not np.any(np.all(a[k][1:] == a[k][:-1], axis=1)), "duplicate cycle"


def full_parity(cc, g, **kw):
    ores = oracle_run(g)
    v, o, hist, lab, front, info = gpu_enumerate(cc, g, **kw)
    assert np.array_equal(hist, ores.hist)
    assert np.array_equal(lab, ores.labels)
    assert np.array_equal(front, ores.front)
    assert_same_cycles(v, o, ores)
    with cc.prepare(g, **kw) as h:
        assert np.array_equal(h.histogram(), ores.hist)
        assert np.array_equal(h.frontier(), ores.front)
        assert h.count() == ores.count
    return info


def four_word_union():
    """256 vertices, ids permuted: two 6x8 grids, two 5x6 grids and C_100."""
    g = gg.disjoint_union(gg.grid(6, 8), gg.grid(6, 8), gg.grid(5, 6), gg.grid(5, 6), gg.cycle(100))
    return gg.permute_random(g, np.random.default_rng(256))


def small_suite():
    rng = np.random.default_rng(4242)
    out = [gg.cycle(3), gg.cycle(4), gg.cycle(64), gg.cycle(65), gg.cycle(128),
           gg.complete(5), gg.complete(12), gg.complete_bipartite(8, 8), gg.wheel(9),
           gg.wheel(64), gg.wheel(100), gg.ladder(20), gg.hypercube(4), gg.hypercube(5),
           gg.complete_multipartite(3, 4, 5), gg.grid(5, 6), gg.grid(6, 6), gg.grid(4, 10),
           gg.permute_random(gg.grid(5, 10), rng), gg.path_graph(30), gg.random_tree(60, rng),
           gg.cone(gg.cycle(20)), gg.disjoint_union(gg.grid(4, 4), gg.wheel(5), gg.complete(4))]
    # More than 128 vertices: four-word bitsets
    out += [gg.cycle(200), gg.cycle(256), gg.wheel(150), gg.cone(gg.cycle(150)),
            gg.disjoint_union(gg.grid(5, 6), gg.grid(6, 6), gg.grid(4, 10), gg.grid(3, 10)),
            gg.permute_random(gg.disjoint_union(gg.grid(6, 8), gg.grid(5, 7), gg.cycle(100)), rng),
            four_word_union()]
    # Sparse enough that the oracle finishes in seconds; n > 64 exercises
    # two-word bitsets.
    for n, m in [(10, 20), (14, 30), (30, 60), (40, 100), (63, 120), (64, 128), (65, 130),
                 (90, 130), (100, 125), (110, 135), (128, 150)]:
        out.append(gg.er_gnm(n, m, np.random.default_rng(4242)))
    return out


@pytest.mark.parametrize("g", small_suite(), ids=lambda g: f"{g.name}_n{g.n}_m{g.m}")
def test_small_suite_parity(cc, g):
    full_parity(cc, g)


@pytest.mark.parametrize("n", [0, 1, 2])
def test_degenerate_sizes(cc, n):
    g = gg.path_graph(n) if n else gg.csr_from_edges(0, [])
    with cc.prepare(g) as h:
        assert h.count() == 0
        assert not h.histogram().any()
        v, o = h.enumerate()
        assert o.numel() == 1 and int(o[0]) == 0


def test_no_edges(cc):
    g = gg.csr_from_edges(50, [])
    with cc.prepare(g) as h:
        assert h.count() == 0 and h.labels().tolist() == list(range(50))


@pytest.mark.parametrize("level", [3, 4, 6, 10])
def test_forced_depth_first_matches(cc, level):
    rng = np.random.default_rng(level)
    for g in [gg.permute_random(gg.grid(5, 7), rng), gg.er_gnm(60, 110, rng),
              gg.er_gnm(100, 125, rng)]:
        info = full_parity(cc, g, force_dfs_level=level)
        assert info["switch_level"] == level


def test_depth_first_steal_heavy_repeated(cc):
    """Regression: a handed-over frontier of a few dozen paths against
    thousands of wavefronts, so nearly all work moves by donation.  Donated
    paths were once read before they were visible on the requester's XCD;
    every repeat must give the oracle's histogram and path counts."""
    rng = np.random.default_rng(4)
    graphs = [gg.permute_random(gg.grid(5, 7), rng), gg.er_gnm(60, 110, rng),
              gg.er_gnm(100, 125, rng)]
    want = [oracle_run(g, cycles=False) for g in graphs]
    for rep in range(6):
        for g, w in zip(graphs, want):
            for level in (4, 5, 7):
                with cc.prepare(g, force_dfs_level=level) as h:
                    assert np.array_equal(h.histogram(), w.hist), (rep, g.name, level)
                    assert np.array_equal(h.frontier(), w.front), (rep, g.name, level)


def test_budget_overflow_switches_to_depth_first(cc):
    # 6x8 grid: the largest level holds 46482 paths; 512 KiB of frontier
    # budget holds about 14600 (enumerate) or 26200 (count) per level, so the
    # levels overflow and hand over to the stacks.
    g = gg.permute_random(gg.grid(6, 8), np.random.default_rng(5))
    info = full_parity(cc, g, budget_bytes=512 << 10)
    assert info["switch_level"] > 3


def test_device_pointer_input(cc):
    import torch
    g = gg.workload_er40()
    rp = torch.tensor(g.row_ptr, dtype=torch.int32, device="cuda")
    ci = torch.tensor(g.col_idx, dtype=torch.int32, device="cuda")
    h = cc.Graph(g.n, rp, ci)
    try:
        assert np.array_equal(h.histogram(), oracle_run(g, cycles=False).hist)
    finally:
        h.release()


def test_host_output_buffers(cc):
    g = gg.grid(5, 6)
    ores = oracle_run(g)
    with cc.prepare(g, output_device=False) as h:
        v, o = h.enumerate()
        assert_same_cycles(v, o, ores)
        # room to spare: one pass, exact sizes returned, the rest untouched
        vb = np.full(ores.n_verts + 1000, -7, np.int32)
        ob = np.full(ores.n_cycles + 50, -7, np.int64)
        nc, nv = h.enumerate_into(vb, ob)
        assert (nc, nv) == (ores.n_cycles, ores.n_verts)
        assert_same_cycles(vb[:nv], ob[:nc + 1], ores)
        assert np.all(vb[nv:] == -7) and np.all(ob[nc + 1:] == -7)
        # too small: the required sizes come back, nothing is written
        vs = np.full(10, -7, np.int32)
        os_ = np.full(3, -7, np.int64)
        with pytest.raises(cc.CCError) as ei:
            h.enumerate_into(vs, os_)
        assert ei.value.status == cc.CC_ERR_BUFFER_TOO_SMALL
        assert ei.value.required == (ores.n_cycles, ores.n_verts)
        assert np.all(vs == -7) and np.all(os_ == -7)


def test_buffer_too_small_reports_sizes(cc):
    import torch
    g = gg.grid(4, 5)
    ores = oracle_run(g)
    with cc.prepare(g) as h:
        v = torch.empty(10, dtype=torch.int32, device="cuda")
        o = torch.empty(3, dtype=torch.int64, device="cuda")
        with pytest.raises(cc.CCError) as ei:
            h.enumerate_into(v, o)
        assert ei.value.status == cc.CC_ERR_BUFFER_TOO_SMALL
        assert ei.value.required == (ores.n_cycles, ores.n_verts)


@pytest.mark.parametrize("case", ["self_loop", "duplicate", "asymmetric", "out_of_range"])
def test_rejects_non_simple(cc, case):
    import torch
    rp, ci = {
        "self_loop": ([0, 2, 3, 4], [0, 1, 0, 0]),
        "duplicate": ([0, 2, 4, 4], [1, 1, 0, 0]),
        "asymmetric": ([0, 1, 1, 1], [1]),
        "out_of_range": ([0, 1, 2, 2], [7, 0]),
    }[case]
    for dev in (False, True):
        r = np.array(rp, np.int32)
        c = np.array(ci, np.int32)
        if dev:
            r = torch.tensor(r, device="cuda")
            c = torch.tensor(c, device="cuda")
        with pytest.raises(cc.CCError) as ei:
            cc.Graph(3, r, c)
        assert ei.value.status == cc.CC_ERR_NOT_SIMPLE


@pytest.mark.parametrize("case", ["first_not_zero", "negative_total", "too_many_entries"])
def test_rejects_invalid_csr_header(cc, case):
    """CSR headers no simple graph on 3 vertices has.  Host arrays are
    rejected before any launch; device arrays by the ingest kernel, which
    answers the host through mapped memory.  A valid graph prepared right
    after each rejection must come out right (the reply words are reused)."""
    import torch
    rp, ci = {
        "first_not_zero": ([1, 2, 3, 4], [1, 0, 0, 0]),
        "negative_total": ([0, 1, 1, -1], [1]),
        "too_many_entries": ([0, 3, 6, 9], [1, 2, 1, 0, 2, 0, 0, 1, 0]),
    }[case]
    tri = gg.complete(3)
    for dev in (False, True):
        r = np.array(rp, np.int32)
        c = np.array(ci, np.int32)
        if dev:
            r = torch.tensor(r, device="cuda")
            c = torch.tensor(c, device="cuda")
        with pytest.raises(cc.CCError) as ei:
            cc.Graph(3, r, c)
        assert ei.value.status == cc.CC_ERR_NOT_SIMPLE
        with cc.prepare(tri) as h:
            assert h.histogram().tolist() == [0, 0, 0, 1]


def test_repeated_runs_identical(cc):
    g = gg.er_gnm(50, 120, np.random.default_rng(3))
    with cc.prepare(g) as h:
        a = [h.histogram() for _ in range(3)]
        assert all(np.array_equal(a[0], x) for x in a)


# ------------------------------------------------------------- workloads
def test_workload_er40_full_enumeration(cc):
    """ER G(40, 100): full enumeration, live oracle."""
    full_parity(cc, gg.workload_er40())


def test_workload_grid8x8_full_enumeration(cc):
    """8x8 grid, ids permuted: full enumeration as int32 vertex lists,
    compared with the stored oracle output."""
    gold = json.load(open(os.path.join(GOLDEN, "grid8x8.json")))
    g = gg.workload_grid8x8()
    v, o, hist, lab, front, info = gpu_enumerate(cc, g)
    assert hist.tolist() == gold["hist"]
    assert lab.tolist() == gold["labels"]
    assert front.tolist() == gold["front"]
    assert int(o[-1]) == gold["total_verts"]
    assert is_canonical_array(v, o)
    assert groups_digest(canonical_groups(v, o)) == gold["canonical_sha256"]


def test_workload_grid8x8_forced_depth_first(cc):
    gold = json.load(open(os.path.join(GOLDEN, "grid8x8.json")))
    g = gg.workload_grid8x8()
    with cc.prepare(g, force_dfs_level=12) as h:
        assert h.histogram().tolist() == gold["hist"]
        assert h.frontier().tolist() == gold["front"]


@pytest.mark.skipif(not os.path.exists(os.path.join(GOLDEN, "grid7x12.json")),
                    reason="stored oracle output for the 7x12 grid not generated")
def test_workload_grid7x12_count_only_4gb(cc):
    """7x12 grid, count-only, 4 GiB frontier budget (the depth-first switch
    is expected to fire)."""
    gold = json.load(open(os.path.join(GOLDEN, "grid7x12.json")))
    g = gg.workload_grid7x12()
    with cc.prepare(g, budget_bytes=4 << 30) as h:
        assert h.histogram().tolist() == gold["hist"]
        assert h.labels().tolist() == gold["labels"]
        assert h.frontier().tolist() == gold["front"]
        info = h.last_run()
        print("grid7x12", info)
    # the frontier outgrows 4 GiB: the levels hand over to the depth-first kernel
    assert info["switch_level"] > 0
    assert info["peak_frontier"] * (8 * 2 + 2) <= 4 << 30


def test_one_level_steps_match(cc):
    """Every breadth-first step one level deep: the same results as the
    default steps, which expand two levels whenever the output fits."""
    full_parity(cc, gg.permute_random(gg.grid(5, 7), np.random.default_rng(8)), one_level_steps=True)
    full_parity(cc, gg.er_gnm(100, 125, np.random.default_rng(8)), one_level_steps=True)
    info = full_parity(cc, gg.permute_random(gg.grid(6, 8), np.random.default_rng(5)),
                       one_level_steps=True, budget_bytes=512 << 10)
    assert info["switch_level"] > 3


# ------------------------------------------------- output by ranges of lengths
def window_groups(cc, g, windows, **kw):
    """Enumerate g window by window (cc_enumerate_lengths); check each
    window's output and return the canonical groups of all of them."""
    groups = {}
    with cc.prepare(g, **kw) as h:
        hist = h.histogram()
        for k0, k1 in windows:
            v, o = h.enumerate_lengths(k0, k1)
            v = v.cpu().numpy() if hasattr(v, "cpu") else v
            o = o.cpu().numpy() if hasattr(o, "cpu") else o
            lens = np.diff(o)
            k = np.arange(hist.size)
            sel = (k >= k0) & (k <= k1)
            assert o[0] == 0 and o.size - 1 == int(hist[sel].sum())
            assert int(o[-1]) == int((hist[sel] * k[sel]).sum())
            assert np.all((lens >= k0) & (lens <= k1)) and np.all(np.diff(lens) >= 0)
            assert is_canonical_array(v, o)
            for kk, a in canonical_groups(v, o).items():
                assert kk not in groups
                groups[kk] = a
    return groups


@pytest.mark.parametrize("case", ["grid5x7", "er60", "er100_w2", "forced_dfs", "host_out"])
def test_length_windows_make_up_the_whole_output(cc, case):
    rng = np.random.default_rng(21)
    g, kw = {
        "grid5x7": (gg.permute_random(gg.grid(5, 7), rng), {}),
        "er60": (gg.er_gnm(60, 110, rng), {}),
        "er100_w2": (gg.er_gnm(100, 125, rng), {}),
        "forced_dfs": (gg.permute_random(gg.grid(5, 7), rng), {"force_dfs_level": 6}),
        "host_out": (gg.er_gnm(40, 100, rng), {"output_device": False}),
    }[case]
    ores = oracle_run(g)
    want = canonical_groups(*ores.cycles)
    windows = [(0, 4), (5, 5), (6, 9), (10, 17), (18, 200)]
    got = window_groups(cc, g, windows, **kw)
    assert sorted(got) == sorted(want)
    for k in want:
        assert np.array_equal(got[k], want[k]), k


def test_length_window_errors_and_pages(cc):
    import torch
    g = gg.permute_random(gg.grid(5, 6), np.random.default_rng(3))
    ores = oracle_run(g)
    hist = ores.hist
    with cc.prepare(g) as h:
        # a window whose buffers are too small reports its own sizes
        k = np.arange(hist.size)
        sel = (k >= 8) & (k <= 12)
        with pytest.raises(cc.CCError) as ei:
            h.enumerate_lengths_into(8, 12, torch.empty(4, dtype=torch.int32, device="cuda"),
                                     torch.empty(2, dtype=torch.int64, device="cuda"))
        assert ei.value.status == cc.CC_ERR_BUFFER_TOO_SMALL
        assert ei.value.required == (int(hist[sel].sum()), int((hist[sel] * k[sel]).sum()))
        with pytest.raises(cc.CCError) as ei:
            h.enumerate_lengths_into(9, 8, torch.empty(4, dtype=torch.int32, device="cuda"),
                                     torch.empty(2, dtype=torch.int64, device="cuda"))
        assert ei.value.status == cc.CC_ERR_INVALID_ARG
        # an empty window: only the closing offset
        v, o = h.enumerate_lengths(200, 300)
        assert o.numel() == 1 and int(o[0]) == 0
        # pages of at most 300 vertex ids cover the whole output
        groups, pages = {}, 0
        biggest = int((hist * k).max())
        for k0, k1, v, o in h.pages(max_verts=max(300, biggest)):
            pages += 1
            assert int(o[-1]) <= max(300, biggest)
            for kk, a in canonical_groups(v.cpu().numpy(), o.cpu().numpy()).items():
                groups[kk] = a
        assert pages > 1
        want = canonical_groups(*ores.cycles)
        assert sorted(groups) == sorted(want)
        assert all(np.array_equal(groups[kk], want[kk]) for kk in want)
        with pytest.raises(ValueError):
            list(h.pages(max_verts=biggest - 1))


# ------------------------------------------------ more than 128 vertices
@pytest.mark.parametrize("level", [3, 5, 9])
def test_four_word_forced_depth_first(cc, level):
    info = full_parity(cc, four_word_union(), force_dfs_level=level)
    assert info["switch_level"] == level


def test_four_word_budget_switch_and_windows(cc):
    g = four_word_union()
    info = full_parity(cc, g, budget_bytes=1 << 20)
    assert info["switch_level"] > 3
    want = canonical_groups(*oracle_run(g).cycles)
    got = window_groups(cc, g, [(0, 6), (7, 12), (13, 300)])
    assert sorted(got) == sorted(want)
    assert all(np.array_equal(got[k], want[k]) for k in want)


def test_too_large_graph_rejected(cc):
    with pytest.raises(cc.CCError) as ei:
        cc.prepare(gg.cycle(1025))
    assert ei.value.status == cc.CC_ERR_TOO_LARGE


def oracle_sorted_list(g, k_min=0, k_max=1 << 30):
    """The oracle's cycles in canonical form, sorted by (k, c0, c1, ...), as
    one flat CSR (written from the oracle's own output, not the HIP path's)."""
    ores = oracle_run(g)
    groups = canonical_groups(*ores.cycles)
    verts, offs = [], [0]
    for k in sorted(groups):
        if k_min <= k <= k_max:
            for row in groups[k]:
                verts.extend(int(x) for x in row)
                offs.append(offs[-1] + k)
    return np.array(verts, np.int64), np.array(offs, np.int64)


@pytest.mark.parametrize("case", ["er40", "grid6x6_host", "forced_dfs", "four_word",
                                  "window", "window_dfs_host"])
def test_sorted_output_equals_sorted_oracle(cc, case):
    """CC_SORTED: the output is exactly the oracle's sorted canonical list,
    element by element (not only as a set), for device and host buffers,
    after a depth-first hand-over (whose cycles arrive in no fixed order),
    with four-word bitsets, and for a window of lengths."""
    import torch
    kw, window = {}, None
    if case == "er40":
        g = gg.workload_er40()
    elif case == "grid6x6_host":
        g = gg.permute_random(gg.grid(6, 6), np.random.default_rng(66))
        kw["output_device"] = False
    elif case == "forced_dfs":
        g = gg.permute_random(gg.grid(5, 7), np.random.default_rng(57))
        kw["force_dfs_level"] = 5
    elif case == "four_word":
        g = four_word_union()
    elif case == "window":
        g = gg.permute_random(gg.grid(5, 8), np.random.default_rng(58))
        window = (6, 12)
    else:
        g = gg.permute_random(gg.grid(5, 8), np.random.default_rng(59))
        kw.update(force_dfs_level=6, output_device=False)
        window = (8, 30)
    with cc.prepare(g, sorted_output=True, **kw) as h:
        if window:
            v, o = h.enumerate_lengths(*window)
        else:
            v, o = h.enumerate()
        if kw.get("output_device", True):
            torch.cuda.synchronize()
            v, o = v.cpu().numpy(), o.cpu().numpy()
    want_v, want_o = oracle_sorted_list(g, *(window or (0, 1 << 30)))
    assert np.array_equal(np.asarray(o, np.int64), want_o)
    assert np.array_equal(np.asarray(v, np.int64)[:want_v.size], want_v)


def test_inputs_written_on_a_side_stream(cc):
    """With no stream given, the binding orders the library's work on torch's
    current stream: a CSR written on a side stream that the current stream
    waits for is seen complete."""
    import torch
    g = gg.workload_er40()
    want = oracle_run(g, cycles=False).hist
    side = torch.cuda.Stream()
    rp = torch.zeros(g.n + 1, dtype=torch.int32, device="cuda")
    ci = torch.zeros(g.col_idx.size, dtype=torch.int32, device="cuda")
    host_rp = torch.tensor(g.row_ptr, dtype=torch.int32).pin_memory()
    host_ci = torch.tensor(g.col_idx, dtype=torch.int32).pin_memory()
    with torch.cuda.stream(side):
        torch.cuda._sleep(2_000_000)  # keep the side stream busy for a while
        rp.copy_(host_rp, non_blocking=True)
        ci.copy_(host_ci, non_blocking=True)
    with torch.cuda.stream(side):
        with cc.Graph(g.n, rp, ci) as h:
            assert np.array_equal(h.histogram(), want)


@pytest.mark.parametrize("case", ["er40", "grid6x7", "k_4_5", "er100_w2", "four_word", "forced_dfs"])
def test_root_ranges_equal_oracle_ranges(cc, case):
    """A range of stage-one roots selects the same cycles, histogram and
    expanded-path counts on the GPU as the oracle's run over that range
    (the oracle numbers roots by u's original id, then x's, then y's)."""
    import torch
    kw = {}
    if case == "er40":
        g = gg.workload_er40()
    elif case == "grid6x7":
        g = gg.permute_random(gg.grid(6, 7), np.random.default_rng(67))
    elif case == "k_4_5":
        g = gg.permute_random(gg.complete_multipartite(4, 5, 3), np.random.default_rng(45))
    elif case == "er100_w2":
        g = gg.er_gnm(100, 150, np.random.default_rng(100))
    elif case == "four_word":
        g = four_word_union()
    else:
        g = gg.permute_random(gg.grid(5, 7), np.random.default_rng(75))
        kw["force_dfs_level"] = 5
    total = oracle.count_roots(g.n, g.row_ptr, g.col_idx)
    rng = np.random.default_rng(7)
    cuts = sorted(set([0, total] + [int(x) for x in rng.integers(0, total + 1, 4)]))
    ranges = list(zip(cuts[:-1], cuts[1:])) + [(0, total), (total // 2, total // 2),
                                                (total - 1, total)]
    with cc.prepare(g, **kw) as h:
        assert h.root_total() == total
        for lo, hi in ranges:
            ores = oracle.enumerate_cycles(g.n, g.row_ptr, g.col_idx, want_cycles=True,
                                           root_lo=lo, root_hi=hi)
            assert np.array_equal(h.histogram_roots(lo, hi), ores.hist), (lo, hi)
            assert np.array_equal(h.frontier(), ores.front), (lo, hi)
            nc, nv = int(ores.hist.sum()), int((ores.hist * np.arange(g.n + 1)).sum())
            v = torch.empty(max(nv, 1), dtype=torch.int32, device="cuda")
            o = torch.empty(nc + 1, dtype=torch.int64, device="cuda")
            assert h.enumerate_roots_into(lo, hi, v, o) == (nc, nv)
            torch.cuda.synchronize()
            assert_same_cycles(v.cpu().numpy()[:nv], o.cpu().numpy(), ores)
        # the whole-graph histogram is still right after range runs
        assert np.array_equal(h.histogram(), oracle_run(g, cycles=False).hist)


@pytest.mark.parametrize("case", ["er40", "grid6x7", "k_4_5", "er100_w2", "four_word", "forced_dfs"])
@pytest.mark.parametrize("out_dev", [True, False])
def test_enumerate_by_roots_groups_equal_oracle_ranges(cc, case, out_dev):
    """The whole output grouped by root in one run: root_first cuts it into
    the oracle's root ranges (each range the same cycle set as the oracle's
    run over it), and the whole is the oracle's cycle set."""
    import torch
    kw = {"output_device": out_dev}
    if case == "er40":
        g = gg.workload_er40()
    elif case == "grid6x7":
        g = gg.permute_random(gg.grid(6, 7), np.random.default_rng(67))
    elif case == "k_4_5":
        g = gg.permute_random(gg.complete_multipartite(4, 5, 3), np.random.default_rng(45))
    elif case == "er100_w2":
        g = gg.er_gnm(100, 150, np.random.default_rng(100))
    elif case == "four_word":
        g = four_word_union()
    else:
        g = gg.permute_random(gg.grid(5, 7), np.random.default_rng(75))
        kw["force_dfs_level"] = 5
    ores = oracle_run(g)
    nc, nv = int(ores.hist.sum()), int((ores.hist * np.arange(g.n + 1)).sum())
    total = oracle.count_roots(g.n, g.row_ptr, g.col_idx)
    with cc.prepare(g, **kw) as h:
        if out_dev:
            v = torch.empty(max(nv, 1), dtype=torch.int32, device="cuda")
            o = torch.empty(nc + 1, dtype=torch.int64, device="cuda")
            f = torch.empty(total + 1, dtype=torch.int64, device="cuda")
        else:
            v, o, f = np.empty(max(nv, 1), np.int32), np.empty(nc + 1, np.int64), np.empty(total + 1, np.int64)
        with pytest.raises(cc.CCError) as ei:
            h.enumerate_by_roots_into(v, o, f[:total])
        assert ei.value.status == cc.CC_ERR_INVALID_ARG
        assert h.enumerate_by_roots_into(v, o, f) == (nc, nv)
        if out_dev:
            torch.cuda.synchronize()
            v, o, f = v.cpu().numpy(), o.cpu().numpy(), f.cpu().numpy()
    assert f[0] == 0 and f[-1] == nc and np.all(np.diff(f) >= 0) and o[-1] == nv
    assert_same_cycles(v[:nv], o, ores, by_length=False)
    for r in range(total):  # each root's cycles ordered by length
        lens = np.diff(o[f[r]:f[r + 1] + 1])
        assert np.all(np.diff(lens) >= 0), r
    rng = np.random.default_rng(11)
    cuts = sorted(set([0, total] + [int(x) for x in rng.integers(0, total + 1, 5)]))
    for lo, hi in list(zip(cuts[:-1], cuts[1:])) + [(total - 1, total), (0, 1)]:
        rres = oracle.enumerate_cycles(g.n, g.row_ptr, g.col_idx, want_cycles=True,
                                       root_lo=lo, root_hi=hi)
        c0, c1 = int(f[lo]), int(f[hi])
        pv, po = v[o[c0]:o[c1]], o[c0:c1 + 1] - o[c0]
        assert_same_cycles(pv, po, rres, by_length=False)


@pytest.mark.parametrize("one_run", [None, True, False])
@pytest.mark.parametrize("out_dev", [True, False])
def test_pages_by_roots_partition_the_output(cc, out_dev, one_run):
    """Pages of consecutive root ranges under a bound: every page fits and
    equals the oracle's run over its roots, and together they are exactly
    the oracle's cycle set (no cycle twice) -- from one grouped run or from
    a run per page."""
    g = gg.permute_random(gg.grid(6, 8), np.random.default_rng(68))
    ores = oracle_run(g)
    nv_all = int((ores.hist * np.arange(g.n + 1)).sum())
    # at least the output of the heaviest single root, else a fraction of all
    total = oracle.count_roots(g.n, g.row_ptr, g.col_idx)
    per_root = [oracle.enumerate_cycles(g.n, g.row_ptr, g.col_idx, want_cycles=False,
                                        root_lo=r, root_hi=r + 1).hist for r in range(total)]
    heaviest = max(int((hr * np.arange(g.n + 1)).sum()) for hr in per_root)
    limit = max(heaviest, nv_all // 7 + 1)
    verts, offs, seen_hi = [], [0], 0
    with cc.prepare(g, output_device=out_dev) as h:
        for lo, hi, v, o in h.pages_by_roots(max_verts=limit, one_run=one_run):
            assert lo == seen_hi and hi > lo
            seen_hi = hi
            v = v.cpu().numpy() if out_dev else np.asarray(v)
            o = o.cpu().numpy() if out_dev else np.asarray(o)
            assert o[-1] <= limit
            rres = oracle.enumerate_cycles(g.n, g.row_ptr, g.col_idx, want_cycles=True,
                                           root_lo=lo, root_hi=hi)
            assert_same_cycles(v[:o[-1]], o, rres, by_length=one_run is False)
            verts.append(v[:o[-1]])
            offs.extend((o[1:] + offs[-1]).tolist())
        assert seen_hi == h.root_total()
    a = canonical_groups(np.concatenate(verts), np.array(offs))
    b = canonical_groups(*ores.cycles)
    assert sorted(a) == sorted(b)
    for k in a:
        assert np.array_equal(a[k], b[k]), k
        if a[k].shape[0] > 1:
            assert not np.any(np.all(a[k][1:] == a[k][:-1], axis=1))
