"""cc_histogram_noalloc (the entry point that allocates nothing: its
workspace is a fixed device array inside the library) against the same
graph through cc_prepare + cc_histogram, called through the C ABI with
device buffers.  Two calls in a row, the second on a smaller graph, so the
second run reuses a workspace the first one left dirty."""
import ctypes

import numpy as np
import pytest

from paper_1410_4876_amd import graphgen as gg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a gfx950 device"
    from paper_1410_4876_amd import cc
    L = cc.lib()
    L.cc_histogram_noalloc.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]
    L.cc_histogram_noalloc.restype = ctypes.c_int
    return torch, cc, L


def noalloc_hist(env, g, extra=3, stream=None):
    torch, cc, L = env
    rp = torch.tensor(g.row_ptr, dtype=torch.int32, device="cuda")
    ci = torch.tensor(g.col_idx if g.col_idx.size else np.zeros(1, np.int32),
                      dtype=torch.int32, device="cuda")
    hist = torch.full((g.n + 1 + extra,), -7, dtype=torch.int64, device="cuda")
    s = stream.cuda_stream if stream is not None else None
    st = L.cc_histogram_noalloc(g.n, rp.data_ptr(), ci.data_ptr(), hist.data_ptr(),
                                hist.numel(), s)
    torch.cuda.synchronize()
    return st, hist.cpu().numpy()


def alloc_hist(env, g):
    torch, cc, L = env
    with cc.prepare(g) as h:
        return h.histogram()


CASES = [
    # a 7x10 grid (two-word bitsets; its frontier outgrows the fixed array, so
    # the depth-first kernel takes over), then ER G(40, 100)
    (lambda: gg.permute_random(gg.grid(7, 10), np.random.default_rng(70)), gg.workload_er40),
    # 256 vertices (four-word bitsets), then a 5x6 grid
    (lambda: gg.permute_random(gg.disjoint_union(gg.grid(6, 8), gg.grid(6, 8), gg.grid(5, 6),
                                                 gg.grid(5, 6), gg.cycle(100)),
                               np.random.default_rng(256)),
     lambda: gg.grid(5, 6)),
    # 1024 vertices (sixteen-word bitsets), then 400 (eight words)
    (lambda: gg.permute_random(gg.tree_plus_edges(1024, 20, np.random.default_rng(3)),
                               np.random.default_rng(33)),
     lambda: gg.tree_plus_edges(400, 18, np.random.default_rng(2))),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_noalloc_matches_cc_histogram_twice(env, case):
    big, small = CASES[case][0](), CASES[case][1]()
    assert small.n < big.n
    for g in (big, small):
        want = alloc_hist(env, g)
        st, got = noalloc_hist(env, g)
        assert st == 0, st
        assert got[:g.n + 1].tolist() == want.tolist(), g.name
        assert (got[g.n + 1:] == 0).all()


def test_noalloc_on_a_side_stream(env):
    torch = env[0]
    g = gg.workload_grid8x8()
    want = alloc_hist(env, g)
    side = torch.cuda.Stream()
    st, got = noalloc_hist(env, g, stream=side)
    assert st == 0 and got[:g.n + 1].tolist() == want.tolist()


def test_noalloc_errors(env):
    torch, cc, L = env
    big = gg.cycle(1025)
    st, _ = noalloc_hist(env, gg.csr_from_edges(3, [(0, 1), (1, 2), (2, 0)]), extra=0)
    assert st == 0
    rp = torch.tensor(big.row_ptr, dtype=torch.int32, device="cuda")
    ci = torch.tensor(big.col_idx, dtype=torch.int32, device="cuda")
    h = torch.zeros(big.n + 1, dtype=torch.int64, device="cuda")
    assert L.cc_histogram_noalloc(big.n, rp.data_ptr(), ci.data_ptr(), h.data_ptr(), h.numel(),
                                  None) == cc.CC_ERR_TOO_LARGE
    g = gg.cycle(6)
    ci_bad = g.col_idx.copy()
    ci_bad[0] = ci_bad[1]  # a repeated neighbour
    bad = gg.CSR(g.n, g.row_ptr, ci_bad, "bad")
    st, _ = noalloc_hist(env, bad)
    assert st == cc.CC_ERR_NOT_SIMPLE
    # hist too short
    rp = torch.tensor(g.row_ptr, dtype=torch.int32, device="cuda")
    ci = torch.tensor(g.col_idx, dtype=torch.int32, device="cuda")
    assert L.cc_histogram_noalloc(g.n, rp.data_ptr(), ci.data_ptr(), h.data_ptr(), g.n,
                                  None) == cc.CC_ERR_INVALID_ARG
    # and a valid call right after the errors still matches
    st, got = noalloc_hist(env, gg.workload_er40())
    assert st == 0 and got[:41].tolist() == alloc_hist(env, gg.workload_er40()).tolist()
