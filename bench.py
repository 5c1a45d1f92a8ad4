#!/usr/bin/env python3
"""Benchmark: chordless cycles/s on one MI355X.

Workload: the 8x8 grid (n=64, m=112, ids permuted with seed 14104876+2),
full enumeration of every chordless cycle as int32 vertex lists into
device buffers.  One step = one whole pass of the path on the resident CSR:
ingest + validation + degree labelling (cc_prepare), stage one, the level
loop and the output (cc_enumerate), and the handle release.

Prints one JSON line with the throughput, the roofline of the dominant
kernel (the breadth-first level kernel, timed with HIP events on the stream
it runs on), and the CPU oracle timed on this host as a baseline.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E, published
PROFILE = os.path.join(ROOT, "profiles", "k_step_grid8x8_enumerate.md")
CSRC = os.path.join(ROOT, "paper_1410_4876_amd", "csrc")
TABLE1 = os.path.join(ROOT, "tests", "golden", "table1.json")
GRID7X12 = os.path.join(ROOT, "tests", "golden", "grid7x12.json")


def library_sources_sha256():
    """sha256 over the library's sources (kernels, their header, the
    runtime that sizes their launches), in name order."""
    import hashlib
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".h")):
            h.update(name.encode())
            h.update(open(os.path.join(CSRC, name), "rb").read())
    return h.hexdigest()


def counted_traffic():
    """HBM bytes per level launch from the committed rocprofv3 PMC summary,
    or None when the library sources have changed since the counters were
    taken."""
    import re
    try:
        text = open(PROFILE).read()
        data = json.loads(re.search(r"```json\n(.*?)\n```", text, re.S).group(1))
        src = library_sources_sha256()
    except (OSError, AttributeError, ValueError):
        return None
    return data["traffic_bytes_per_launch"] if data.get("library_sources_sha256") == src else None


def cpu_baseline(g, budget_s=30.0):
    """The oracle (single thread, one counting+storing pass) on the same
    graph.  The 8x8 grid takes about 15 s, inside the bounded budget."""
    import oracle
    t0 = time.perf_counter()
    r = oracle.enumerate_single_pass(g.n, g.row_ptr, g.col_idx, verts_cap=64 << 20,
                                     cyc_cap=4 << 20)
    dt = time.perf_counter() - t0
    return {"value": round(r.n_cycles / dt, 1), "unit": "chordless cycles/s", "cores": 1,
            "kind": "oracle",
            "sample": f"whole workload, one pass storing all cycles ({r.n_cycles} cycles, "
                      f"{dt:.1f} s, single thread)"}


def batched_section(args):
    """4096 ER graphs (n in [16, 64], d in [2.5, 5]): per-graph histograms
    with one persistent launch (autotuned on a held-out calibration batch)
    against the same kernels launched once per graph."""
    import torch

    from paper_1410_4876_amd import autotune, cc
    from paper_1410_4876_amd import graphgen as gg

    tuned = autotune.tune_batch()
    b = gg.workload_batch4096()
    with cc.prepare_batch(b, **tuned["options"]) as h:
        h.histograms()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            hist = h.histograms()
        dt = (time.perf_counter() - t0) / args.steps
        cycles = int(hist.sum())
        paths = h.last_run()["paths"]
        t0 = time.perf_counter()
        hist_pg = h.histograms(per_graph_launch=True)
        dt_pg = time.perf_counter() - t0
        launches_pg = h.last_run()["levels_launched"]
    assert np.array_equal(hist, hist_pg)
    return {"workload": "4096 ER graphs, n in [16,64], d in [2.5,5]", "cycles": cycles,
            "paths_expanded": int(paths),
            "persistent": {"ms": round(dt * 1e3, 3), "cycles_per_s": round(cycles / dt, 1),
                           "launches": 3},
            "per_graph_launch": {"ms": round(dt_pg * 1e3, 3),
                                 "cycles_per_s": round(cycles / dt_pg, 1),
                                 "launches": int(launches_pg)},
            "speedup": round(dt_pg / dt, 2),
            "autotuned": tuned["options"], "autotune_calibration_ms": tuned["ms"]}


def table1_section(args):
    """Table 1's structured graphs (Section 5): the counts, which must equal
    the printed ones, and MI355X times in the paper's two forms.  proc: CSR
    resident on the device, prepare (ingest + labelling) and enumeration
    into device buffers.  total: CSR from host memory, results copied back
    into host buffers.  Grid 8x10 is count-only, as in the paper.  Median
    and mean of 10 runs after 3 warm-ups; the paper's R9 290X times are
    context, not a target."""
    import torch

    from paper_1410_4876_amd import cc
    from paper_1410_4876_amd import graphgen as gg

    rows = json.load(open(TABLE1))["rows"]
    out = []
    for r in rows:
        g = getattr(gg, r["family"])(*r["args"])
        rp = torch.tensor(g.row_ptr, dtype=torch.int32, device="cuda")
        ci = torch.tensor(g.col_idx, dtype=torch.int32, device="cuda")
        with cc.Graph(g.n, rp, ci) as h:
            hist = h.histogram()
        assert int(hist[3]) == r["c3"] and int(hist[4:].sum()) == r["clc"], r["name"]
        nc = int(hist.sum())
        nv = int((hist * np.arange(hist.size)).sum())
        dv = torch.empty(max(nv, 1), dtype=torch.int32, device="cuda")
        do = torch.empty(nc + 1, dtype=torch.int64, device="cuda")
        hv = np.empty(max(nv, 1), np.int32)
        ho = np.empty(nc + 1, np.int64)

        def proc():
            with cc.Graph(g.n, rp, ci) as h:
                if r["count_only"]:
                    h.count()
                else:
                    h.enumerate_into(dv, do)
            torch.cuda.synchronize()

        def total():
            with cc.Graph(g.n, g.row_ptr, g.col_idx, output_device=False) as h:
                if r["count_only"]:
                    h.histogram()
                else:
                    h.enumerate_into(hv, ho)
            torch.cuda.synchronize()

        def timed(fn):
            for _ in range(3):
                fn()
            ts = []
            for _ in range(10):
                t0 = time.perf_counter()
                fn()
                ts.append((time.perf_counter() - t0) * 1e3)
            return float(np.median(ts)), float(np.mean(ts))

        p_med, p_mean = timed(proc)
        t_med, t_mean = timed(total)
        out.append({"name": r["name"], "n": r["n"], "m": r["m"], "c3": r["c3"], "clc": r["clc"],
                    "count_only": r["count_only"],
                    "proc_ms": {"median": round(p_med, 4), "mean": round(p_mean, 4)},
                    "total_ms": {"median": round(t_med, 4), "mean": round(t_mean, 4)},
                    "paper_r9_290x_ms": {"proc": r["t_par_proc_ms"], "total": r["t_par_total_ms"]},
                    "proc_speedup_vs_paper": round(r["t_par_proc_ms"] / p_mean, 1)})
    return {"rows": out, "counts_equal_table1": True}


def _timed(fn, warmup=3, runs=10):
    """Median and mean wall ms of `runs` calls after `warmup` untimed ones."""
    for _ in range(warmup):
        fn()
    ts = []
    for _ in range(runs):
        t0 = time.perf_counter()
        fn()
        ts.append((time.perf_counter() - t0) * 1e3)
    return {"median": round(float(np.median(ts)), 4), "mean": round(float(np.mean(ts)), 4)}


def er40_section():
    """ER G(40, 100), full enumeration: a latency-bound call.  proc: CSR on
    the device, results into device buffers; total: CSR from host memory,
    results copied into host buffers."""
    import torch

    from paper_1410_4876_amd import cc
    from paper_1410_4876_amd import graphgen as gg

    g = gg.workload_er40()
    rp = torch.tensor(g.row_ptr, dtype=torch.int32, device="cuda")
    ci = torch.tensor(g.col_idx, dtype=torch.int32, device="cuda")
    with cc.Graph(g.n, rp, ci) as h:
        hist = h.histogram()
    nc = int(hist.sum())
    nv = int((hist * np.arange(hist.size)).sum())
    dv = torch.empty(max(nv, 1), dtype=torch.int32, device="cuda")
    do = torch.empty(nc + 1, dtype=torch.int64, device="cuda")
    hv = np.empty(max(nv, 1), np.int32)
    ho = np.empty(nc + 1, np.int64)

    def proc():
        with cc.Graph(g.n, rp, ci) as h:
            h.enumerate_into(dv, do)
        torch.cuda.synchronize()

    def total():
        with cc.Graph(g.n, g.row_ptr, g.col_idx, output_device=False) as h:
            h.enumerate_into(hv, ho)

    p = _timed(proc)
    return {"workload": "ER G(40,100), seed index 1, full enumeration", "cycles": nc,
            "proc_ms": p, "total_ms": _timed(total),
            "cycles_per_s": round(nc / (p["median"] * 1e-3), 1)}


def grid7x12_section():
    """7x12 grid (n=84, m=149), ids permuted, count-only with an int64
    per-length histogram and a 4 GiB frontier budget: the levels hand over
    to the depth-first kernel.  The histogram must equal the stored oracle
    output.  Reports the switch, the peak frontier, and each phase."""
    import torch

    from paper_1410_4876_amd import cc
    from paper_1410_4876_amd import graphgen as gg

    gold = json.load(open(GRID7X12))
    g = gg.workload_grid7x12()
    rp = torch.tensor(g.row_ptr, dtype=torch.int32, device="cuda")
    ci = torch.tensor(g.col_idx, dtype=torch.int32, device="cuda")
    budget = 4 << 30

    def run(profile=False):
        with cc.Graph(g.n, rp, ci, budget_bytes=budget, profile=profile) as h:
            hist = h.histogram()
            return hist, h.frontier(), h.last_run()

    hist, front, _ = run()
    assert hist.tolist() == gold["hist"] and front.tolist() == gold["front"]
    t = _timed(lambda: run())
    _, _, info = run(profile=True)
    cycles, paths = int(hist.sum()), int(front.sum())
    lvl = info["level_ms"] + info["head_ms"]
    lvl_bytes = info["level_bytes"] + info["head_bytes"]
    w_bytes = 8 * 2 + 2  # W=2 words of X plus the two end labels, per path
    return {"workload": "grid 7x12 (n=84, m=149), ids permuted, count-only, 4 GiB frontier budget",
            "cycles": cycles, "paths_expanded": paths, "ms": t,
            "cycles_per_s": round(cycles / (t["median"] * 1e-3), 1),
            "paths_per_s": round(paths / (t["median"] * 1e-3), 1),
            "switch_level": info["switch_level"],
            "peak_frontier_paths": info["peak_frontier"],
            "peak_frontier_bytes": info["peak_frontier"] * w_bytes,
            "breadth_first": {"ms": round(lvl, 4), "bytes": lvl_bytes,
                              "GBps": round(lvl_bytes / (lvl * 1e-3) / 1e9, 1) if lvl > 0 else 0.0,
                              "hbm_frac": round(lvl_bytes / (lvl * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)
                              if lvl > 0 else 0.0},
            "depth_first": {"ms": round(info["dfs_ms"], 4),
                            "paths_per_s": round(
                                (paths - int(front[:info["switch_level"]].sum()))
                                / (info["dfs_ms"] * 1e-3), 1) if info["dfs_ms"] > 0 else 0.0},
            "stage1_ms": round(info["stage1_ms"], 4)}


def paging_section():
    """Grid 7x10 (8,136,453 cycles, 0.95 GB of vertex ids): the whole output
    in one cc_enumerate call, and the same output paged through buffers of
    at most 64 Mi vertex ids (256 MiB) by ranges of cycle lengths
    (cc_enumerate_lengths).  Every page reruns the enumeration."""
    import torch

    from paper_1410_4876_amd import cc
    from paper_1410_4876_amd import graphgen as gg

    g = gg.grid(7, 10)
    rp = torch.tensor(g.row_ptr, dtype=torch.int32, device="cuda")
    ci = torch.tensor(g.col_idx, dtype=torch.int32, device="cuda")
    limit = 64 << 20
    with cc.Graph(g.n, rp, ci) as h:
        hist = h.histogram()
        nc = int(hist.sum())
        nv = int((hist * np.arange(hist.size)).sum())
        dv = torch.empty(nv, dtype=torch.int32, device="cuda")
        do = torch.empty(nc + 1, dtype=torch.int64, device="cuda")

        def whole():
            h.enumerate_into(dv, do)
            torch.cuda.synchronize()

        def paged():
            pages = 0
            for _, _, v, o in h.pages(max_verts=limit):
                pages += 1
            torch.cuda.synchronize()
            return pages

        w = _timed(whole, warmup=2, runs=5)
        pages = paged()
        p = _timed(paged, warmup=1, runs=3)
    return {"workload": "grid 7x10, full enumeration", "cycles": nc, "vertex_ids": nv,
            "whole_ms": w, "page_limit_vertex_ids": limit, "pages": pages, "paged_ms": p}


def large_n_section():
    """Graphs of more than 128 vertices (four-word bitsets), full enumeration
    with CSR and results on the device: C_256, and 256 vertices made of two
    6x8 grids, two 5x6 grids and C_100 with ids permuted."""
    import torch

    from paper_1410_4876_amd import cc
    from paper_1410_4876_amd import graphgen as gg

    union = gg.permute_random(gg.disjoint_union(gg.grid(6, 8), gg.grid(6, 8), gg.grid(5, 6),
                                                gg.grid(5, 6), gg.cycle(100)),
                              np.random.default_rng(256))
    out = []
    for g in [gg.cycle(256), union]:
        rp = torch.tensor(g.row_ptr, dtype=torch.int32, device="cuda")
        ci = torch.tensor(g.col_idx, dtype=torch.int32, device="cuda")
        with cc.Graph(g.n, rp, ci) as h:
            hist = h.histogram()
        nc = int(hist.sum())
        nv = int((hist * np.arange(hist.size)).sum())
        dv = torch.empty(max(nv, 1), dtype=torch.int32, device="cuda")
        do = torch.empty(nc + 1, dtype=torch.int64, device="cuda")

        def proc():
            with cc.Graph(g.n, rp, ci) as h:
                h.enumerate_into(dv, do)
            torch.cuda.synchronize()

        t = _timed(proc)
        out.append({"graph": g.name, "n": g.n, "m": g.m, "cycles": nc, "proc_ms": t,
                    "cycles_per_s": round(nc / (t["median"] * 1e-3), 1)})
    return {"rows": out}


def serving_section(args):
    """Open-loop Poisson request stream (2000 requests/s; half p x q grids,
    p, q in 3..7, half ER graphs, n in 20..80, d in [3, 5]) replayed against
    the serving loop; p50/p99 latency beside throughput."""
    from paper_1410_4876_amd import cc, loadgen
    from paper_1410_4876_amd import graphgen as gg

    reqs = gg.request_stream(rate_hz=2000.0, duration_s=args.serve_seconds, k=5)
    with cc.Server() as sv:
        # warm-up: a short stream of its own, not part of the figures
        loadgen.run_stream(sv, gg.request_stream(rate_hz=2000.0, duration_s=0.2, k=1005))
        r = loadgen.run_stream(sv, reqs)
    out = {k: v for k, v in r.items() if k not in ("hists", "statuses")}
    out["workload"] = (f"Poisson stream at 2000 requests/s for {args.serve_seconds:g} s: "
                       "grids p x q (p, q in 3..7) and ER graphs (n in 20..80, d in [3,5]), "
                       "ids permuted")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only time a plain 1 GiB device-to-device copy (counter calibration)")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the 4096-graph batched vs per-graph-launch comparison")
    ap.add_argument("--serve-seconds", type=float, default=5.0,
                    help="length of the replayed request stream (the full stream is 60 s)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving stream")
    ap.add_argument("--no-table1", action="store_true",
                    help="skip the structured graphs of the paper's Table 1")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the ER G(40,100) latency, 7x12 count-only and paging sections")
    ap.add_argument("--section",
                    choices=["er40", "grid7x12", "paging", "large_n", "table1", "batched",
                             "serving"],
                    help="run only this section and print its JSON (for profiling one workload)")
    ap.add_argument("--no-profile", action="store_true",
                    help="time steps without per-kernel HIP events (no roofline)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; the path shards by triplet "
                                   "or by graph across GPUs, which is not built here",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    from paper_1410_4876_amd import cc
    from paper_1410_4876_amd import graphgen as gg

    torch.cuda.set_device(0)
    if args.section:
        fn = {"er40": er40_section, "grid7x12": grid7x12_section, "paging": paging_section,
              "large_n": large_n_section,
              "table1": lambda: table1_section(args), "batched": lambda: batched_section(args),
              "serving": lambda: serving_section(args)}[args.section]
        print(json.dumps({args.section: fn()}), flush=True)
        return
    if args.calibrate_copy:
        # A plain copy of known size: what the HBM byte counters read for it
        # scales the counters read for the level kernel.
        src = torch.ones(1 << 28, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(args.warmup):
            dst.copy_(src)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            dst.copy_(src)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / max(args.steps, 1)
        print(json.dumps({"copy_bytes_read": src.numel() * 4, "copy_bytes_written": src.numel() * 4,
                          "ms": round(dt * 1e3, 4),
                          "GBps_read_plus_write": round(2 * src.numel() * 4 / dt / 1e9, 1)}))
        return
    g = gg.workload_grid8x8()
    rp = torch.tensor(g.row_ptr, dtype=torch.int32, device="cuda")
    ci = torch.tensor(g.col_idx, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    profile = not args.no_profile

    # exact output sizes (outside the timed region)
    with cc.Graph(g.n, rp, ci, stream=stream) as h0:
        hist = h0.histogram()
    n_cycles = int(hist.sum())
    n_verts = int((hist * np.arange(hist.size)).sum())
    verts = torch.empty(n_verts, dtype=torch.int32, device="cuda")
    offs = torch.empty(n_cycles + 1, dtype=torch.int64, device="cuda")

    def step(profile, persistent_levels=False):
        with cc.Graph(g.n, rp, ci, stream=stream, profile=profile,
                      persistent_levels=persistent_levels) as h:
            nc, nv = h.enumerate_into(verts, offs)
            assert nc == n_cycles and nv == n_verts
            return h.last_run()

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = [step(False) for _ in range(args.steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed * 1e3 / args.steps

    out = {
        "metric": "chordless cycles/s on 1 MI355X",
        "value": round(n_cycles * args.steps / elapsed, 1),
        "unit": "chordless cycles/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64", "data": "synthetic",
        "config": {"workload": "grid 8x8 (n=64, m=112), ids permuted, full enumeration to "
                               "int32 vertex lists", "cycles": n_cycles, "vertices_out": n_verts,
                   "paths_expanded": int(infos[-1]["paths"]), "parallelism": "single GPU"},
        "paths_per_s": round(infos[-1]["paths"] * args.steps / elapsed, 1),
        "gpu_ms_per_step": round(sum(i["gpu_ms"] for i in infos) / len(infos), 4),
    }
    if profile:
        # Second timed pass of the same steps with HIP event pairs around
        # every breadth-first step launch (on the stream the kernels run on):
        # the step kernel's average launch duration and the bytes it must
        # move.
        torch.cuda.synchronize()
        pinfos = [step(True) for _ in range(args.steps)]
        torch.cuda.synchronize()
        lvl_ms = sum(i["level_ms"] for i in pinfos)
        lvl_bytes = sum(i["level_bytes"] for i in pinfos)
        launches = sum(i["levels_launched"] for i in pinfos)
        achieved = lvl_bytes / (lvl_ms * 1e-3) / 1e9 if lvl_ms > 0 else 0.0
        persistent = launches == len(pinfos)
        out["roofline"] = {"bound": "hbm",
                           "kernel": ("k_levels (all breadth-first steps in one cooperative "
                                      "launch)" if persistent else
                                      "k_step (breadth-first step: one or two levels per "
                                      "launch, staged-cycle decode)"),
                           "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                           "frac": round(achieved / HBM_PEAK_GBPS, 4),
                           "traffic": counted_traffic(),
                           "bytes_per_launch": round(lvl_bytes / max(launches, 1), 1),
                           "avg_launch_us": round(lvl_ms * 1e3 / max(launches, 1), 3),
                           "launches_per_step": round(launches / len(pinfos), 1),
                           "measured": "HIP events around every step launch, second pass of "
                                       "the timed steps"}
        out["breakdown_ms"] = {
            "stage1": round(sum(i["stage1_ms"] for i in pinfos) / len(pinfos), 4),
            "head": round(sum(i["head_ms"] for i in pinfos) / len(pinfos), 4),
            "levels": round(lvl_ms / len(pinfos), 4),
            "dfs": round(sum(i["dfs_ms"] for i in pinfos) / len(pinfos), 4)}
        out["head_steps"] = pinfos[-1]["head_steps"]
        # the same step with all levels in one cooperative launch, for comparison
        for _ in range(2):
            step(False, persistent_levels=True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            step(False, persistent_levels=True)
        torch.cuda.synchronize()
        out["persistent_level_loop_ms_per_step"] = round(
            (time.perf_counter() - t1) * 1e3 / args.steps, 4)
    if not args.no_batch:
        out["batched"] = batched_section(args)
    if not args.no_serve:
        out["serving"] = serving_section(args)
    if not args.no_extra:
        out["er40"] = er40_section()
        out["grid7x12"] = grid7x12_section()
        out["paging"] = paging_section()
        out["large_n"] = large_n_section()
    if not args.no_table1:
        out["table1"] = table1_section(args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(g)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
