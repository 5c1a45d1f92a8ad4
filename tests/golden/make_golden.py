"""Writes the stored expected values for workloads too large to run through
the oracle inside the test suite.  Calls only the CPU oracle (plus the input
generators); nothing here touches the HIP path.

    python tests/golden/make_golden.py grid7x12   # ~10 min on 8 cores
    python tests/golden/make_golden.py grid8x8    # ~40 s, one core
    python tests/golden/make_golden.py batch4096
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1410_4876_amd import graphgen as gg  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def grid7x12(procs):
    g = gg.workload_grid7x12()
    t = time.time()
    hist, front = oracle.histogram_parallel(g.n, g.row_ptr, g.col_idx, procs=procs,
                                            splits=512)
    out = {
        "workload": "7x12 grid (n=84, m=149), ids permuted with seed 14104876+3",
        "made_by": "tests/golden/make_golden.py grid7x12 (CPU oracle only)",
        "n": g.n, "m": g.m,
        "labels": oracle.degree_labelling(g.n, g.row_ptr, g.col_idx).tolist(),
        "hist": hist.tolist(), "front": front.tolist(),
        "total_cycles": int(hist.sum()), "total_paths": int(front.sum()),
        "oracle_seconds": round(time.time() - t, 1), "procs": procs,
    }
    with open(os.path.join(HERE, "grid7x12.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({k: v for k, v in out.items() if k not in ("hist", "front", "labels")}))


def grid8x8(procs):
    sys.path.insert(0, os.path.dirname(HERE))
    from ccutil import canonical_groups, groups_digest
    g = gg.workload_grid8x8()
    t = time.time()
    r = oracle.enumerate_cycles(g.n, g.row_ptr, g.col_idx, want_cycles=True)
    verts, offs = r.cycles
    groups = canonical_groups(verts, offs)
    out = {
        "workload": "8x8 grid (n=64, m=112), ids permuted with seed 14104876+2",
        "made_by": "tests/golden/make_golden.py grid8x8 (CPU oracle only)",
        "n": g.n, "m": g.m,
        "labels": r.labels.tolist(), "hist": r.hist.tolist(), "front": r.front.tolist(),
        "total_cycles": int(r.hist.sum()), "total_paths": int(r.front.sum()),
        "total_verts": int(r.n_verts),
        "canonical_sha256": groups_digest(groups),
        "oracle_seconds": round(time.time() - t, 1), "procs": 1,
    }
    with open(os.path.join(HERE, "grid8x8.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({k: v for k, v in out.items() if k not in ("hist", "front", "labels")}))


def _one(args):
    n, rp, ci = args
    r = oracle.enumerate_cycles(n, rp, ci, want_cycles=False)
    return r.hist, r.front


def batch4096(procs):
    import multiprocessing as mp
    b = gg.workload_batch4096()
    t = time.time()
    jobs = [(g.n, g.row_ptr, g.col_idx) for g in b.graphs]
    with mp.get_context("fork").Pool(procs) as pool:
        res = pool.map(_one, jobs, chunksize=4)
    hists = [h.tolist() for h, _ in res]
    out = {
        "workload": "4096 ER graphs, n in [16,64], d in [2.5,5], m=floor(n*d/2+0.5), seed 14104876+4",
        "made_by": "tests/golden/make_golden.py batch4096 (CPU oracle only)",
        "hists": hists,
        "total_cycles": int(sum(sum(h) for h in hists)),
        "total_paths": int(sum(int(f.sum()) for _, f in res)),
        "oracle_seconds": round(time.time() - t, 1), "procs": procs,
    }
    with open(os.path.join(HERE, "batch4096.json"), "w") as f:
        json.dump(out, f, separators=(",", ":"))
    print(json.dumps({k: v for k, v in out.items() if k != "hists"}))


if __name__ == "__main__":
    which = sys.argv[1]
    procs = int(sys.argv[2]) if len(sys.argv) > 2 else (os.cpu_count() or 1)
    {"grid7x12": grid7x12, "grid8x8": grid8x8, "batch4096": batch4096}[which](procs)
