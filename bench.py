#!/usr/bin/env python3
"""Benchmark: chordless cycles/s on one MI355X, batched vs per-graph launch.

Headline workload: 4096 Erdos-Renyi graphs (n uniform in [16, 64], average
degree uniform in [2.5, 5], seed 14104876+4), packed as one int32 CSR that is
resident in device memory.  One step = one whole pass of the path over the
batch: ingest + validation + degree labelling of every graph
(cc_prepare_batch), stage one and the persistent depth-first launch with
work stealing (cc_histogram_batch, count-only per-graph histograms), and the
handle release.  The result of the timed steps must equal the stored oracle
histograms.  Two per-graph baselines run the same workload: the same kernels
launched once per graph on the same full grid, and one cc_prepare +
cc_histogram call per graph.

Prints one JSON line with the throughput, the roofline of the dominant
kernel (the batched depth-first kernel, timed with HIP events on the stream
it runs on), the CPU oracle timed on this host as a baseline, and the other
workloads (8x8 grid enumeration, 7x12 grid count-only, ER G(40,100), the
serving stream, the paper's Table 1 graphs).
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
# LDS bandwidth from unit counts: 256 CUs x 128 bytes per clock x 2.4 GHz
LDS_PEAK_GBPS = 256 * 128 * 2.4
PROFILES = os.path.join(ROOT, "profiles")
TABLE1 = os.path.join(ROOT, "tests", "golden", "table1.json")
GRID7X12 = os.path.join(ROOT, "tests", "golden", "grid7x12.json")
GRID8X8 = os.path.join(ROOT, "tests", "golden", "grid8x8.json")
BATCH4096 = os.path.join(ROOT, "tests", "golden", "batch4096.json")
BATCH_WORKLOAD = ("4096 ER graphs, n uniform in [16,64], average degree uniform in [2.5,5], "
                  "one packed int32 CSR resident on the device; count-only per-graph histograms")
# Algorithmic bytes per path processed by the depth-first kernel, count-only
# with W-word bitsets: the rows N(vt) and N(v1) read (16W), and the path
# state (X words, v1, vt) pushed once and popped once (2 * (8W + 2)).
def dfs_bytes_per_path(W):
    return 16 * W + 2 * (8 * W + 2)


def counted_traffic(profile_name):
    """HBM bytes per launch from a committed rocprofv3 PMC summary, or None
    when the library sources have changed since the counters were taken."""
    import re

    from paper_1410_4876_amd.build import sources_sha256
    try:
        text = open(os.path.join(PROFILES, profile_name)).read()
        data = json.loads(re.search(r"```json\n(.*?)\n```", text, re.S).group(1))
    except (OSError, AttributeError, ValueError):
        return None
    return (data["traffic_bytes_per_launch"]
            if data.get("library_sources_sha256") == sources_sha256() else None)


# ------------------------------------------------------------ CPU baseline
def _cpu_info():
    procs = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    # at most 16 workers: the share of host cores that goes with one GPU
    return {"nproc": int(procs or 1), "workers": int(min(16, procs or 1)), "model": model}


def _oracle_graph(args):
    import oracle
    n, rp, ci, lo, hi = args
    r = oracle.enumerate_cycles(n, rp, ci, want_cycles=False, root_lo=lo, root_hi=hi)
    return int(r.hist.sum()), int(r.front.sum())


def _bounded(jobs, workers, budget_s):
    """Runs oracle jobs (graph, root range) in order until the time budget
    is spent: in this process for one worker, else on a process pool
    (forked before this process touches the GPU) with one job in flight per
    worker.  Jobs already started when the budget runs out get up to
    another budget to finish; any still running then are abandoned and
    their work is not counted (the rate is then a lower bound).  Returns
    (cycles, paths, jobs done, seconds, jobs abandoned)."""
    import multiprocessing as mp
    import queue
    t0 = time.perf_counter()
    cyc = paths = done = 0
    if workers == 1:
        for j in jobs:
            c, p = _oracle_graph(j)
            cyc, paths, done = cyc + c, paths + p, done + 1
            if time.perf_counter() - t0 > budget_s:
                break
        return cyc, paths, done, time.perf_counter() - t0, 0
    ctx = mp.get_context("fork")
    results = queue.Queue()
    it = iter(jobs)
    pool = ctx.Pool(workers)
    try:
        inflight = 0
        for _ in range(workers):
            j = next(it, None)
            if j is None:
                break
            pool.apply_async(_oracle_graph, (j,), callback=results.put)
            inflight += 1
        while inflight:
            left = 2 * budget_s - (time.perf_counter() - t0)
            if left <= 0:
                break
            try:
                c, p = results.get(timeout=left)
            except queue.Empty:
                break
            inflight -= 1
            cyc, paths, done = cyc + c, paths + p, done + 1
            if time.perf_counter() - t0 <= budget_s:
                j = next(it, None)
                if j is not None:
                    pool.apply_async(_oracle_graph, (j,), callback=results.put)
                    inflight += 1
        dt = time.perf_counter() - t0
    finally:
        pool.terminate()
        pool.join()
    return cyc, paths, done, dt, inflight


def cpu_baselines(budget_s):
    """The oracle as it stands, timed on this host's cores on bounded samples
    of every config (run before the process touches the GPU).  Returns the
    headline's baseline (the 4096-graph batch on all workers) and the
    per-config table."""
    import oracle
    from paper_1410_4876_amd import graphgen as gg

    info = _cpu_info()
    W = info["workers"]
    out = {"host": info}

    def rate(res, cores, what):
        c, p, d, dt, ab = res
        note = f", {ab} started but unfinished, not counted" if ab else ""
        return {"cycles_per_s": round(c / dt, 1), "paths_per_s": round(p / dt, 1),
                "jobs_per_s": round(d / dt, 2), "cores": cores,
                "sample": f"{d} {what} done in {dt:.1f} s{note}"}

    b = gg.workload_batch4096()
    jobs = [(g.n, g.row_ptr, g.col_idx, 0, oracle.INT64_MAX) for g in b.graphs]
    out["batch4096_single_thread"] = rate(_bounded(jobs, 1, budget_s), 1,
                                          "graphs (in order from graph 0)")
    out["batch4096_all_cores"] = rate(_bounded(jobs, W, budget_s), W,
                                      "graphs (in order from graph 0, one per worker at a time)")
    g = gg.workload_er40()
    t0 = time.perf_counter()
    r = oracle.enumerate_single_pass(g.n, g.row_ptr, g.col_idx, verts_cap=1 << 22, cyc_cap=1 << 20)
    dt = time.perf_counter() - t0
    out["er40_single_thread"] = {"cycles_per_s": round(r.n_cycles / dt, 1), "cores": 1,
                                 "sample": f"whole graph, cycles stored, {dt * 1e3:.1f} ms"}

    def root_jobs(g, chunks):
        roots = oracle.count_roots(g.n, g.row_ptr, g.col_idx)
        bounds = np.linspace(0, roots, min(chunks, roots) + 1).astype(np.int64)
        return [(g.n, g.row_ptr, g.col_idx, int(bounds[i]), int(bounds[i + 1]))
                for i in range(len(bounds) - 1)]

    out["grid8x8_single_thread"] = rate(_bounded(root_jobs(gg.workload_grid8x8(), 64), 1,
                                                 budget_s / 2), 1,
                                        "of 64 initial-triplet ranges (count-only)")
    out["grid7x12_all_cores"] = rate(_bounded(root_jobs(gg.workload_grid7x12(), 512), W,
                                              budget_s / 2), W,
                                     "single initial triplets (count-only)")
    reqs = gg.request_stream(rate_hz=2000.0, duration_s=5.0, k=5)
    jobs = [(r.graph.n, r.graph.row_ptr, r.graph.col_idx, 0, oracle.INT64_MAX) for r in reqs]
    out["serving_requests_all_cores"] = rate(_bounded(jobs, W, budget_s / 2), W,
                                             "requests (in arrival order)")
    head = out["batch4096_all_cores"]
    return {"value": head["cycles_per_s"], "unit": "chordless cycles/s", "cores": W,
            "kind": "oracle", "sample": "4096-graph batch: " + head["sample"],
            "per_config": out}


# ------------------------------------------------------------ headline
def _batch_device(b):
    import torch
    return (torch.tensor(b.graph_vtx_off, dtype=torch.int32, device="cuda"),
            torch.tensor(b.row_ptr, dtype=torch.int32, device="cuda"),
            torch.tensor(b.col_idx, dtype=torch.int32, device="cuda"))


def _dfs_diag(info):
    """What the depth-first kernel's wavefronts did: steps, the share of
    lanes that held a path, the share of time spent looking for work."""
    return {"steps": int(info["dfs_steps"]), "lane_use": round(info["dfs_lane_use"], 4),
            "idle_frac": round(info["dfs_idle_frac"], 4), "donations": int(info["dfs_donations"]),
            "fills": int(info["dfs_fills"]), "spilled_entries": int(info["dfs_spills"]),
            "global_hist_adds": int(info["dfs_global_adds"])}


def batched_headline(args, baselines=True):
    """The 4096-graph batch: whole passes (prepare + persistent histogram +
    release) on the resident CSR, autotuned launch options, HIP events
    around the depth-first kernel; then the two per-graph baselines.  Every
    result must equal the stored oracle histograms."""
    import torch

    from paper_1410_4876_amd import autotune, cc
    from paper_1410_4876_amd import graphgen as gg

    gold = json.load(open(BATCH4096))
    tuned = autotune.tune_batch()
    opts = tuned["options"]
    b = gg.workload_batch4096()
    G = len(b.graphs)
    sizes = np.diff(np.asarray(b.graph_vtx_off, np.int64))
    hoff = np.zeros(G, np.int64)
    hoff[1:] = np.cumsum(sizes + 1)[:-1]
    total = int((sizes + 1).sum())
    off_d, rp_d, ci_d = _batch_device(b)
    stream = torch.cuda.current_stream()

    def check(buf, what):
        for g in range(G):
            want = gold["hists"][g]
            got = buf[hoff[g]:hoff[g] + sizes[g] + 1]
            assert got[:len(want)].tolist() == want and not got[len(want):].any(), (what, g)

    buf = np.zeros(total, np.int64)
    infos = []

    def step():
        with cc.Batch(off_d, rp_d, ci_d, stream=stream, sizes=sizes, profile=True, **opts) as h:
            h.histograms_into(buf, hoff)
            infos.append(h.last_run())

    for _ in range(args.warmup):
        step()
    infos.clear()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    check(buf, "persistent")
    cycles = int(gold["total_cycles"])
    paths = int(infos[-1]["paths"])
    assert paths == gold["total_paths"] and int(infos[-1]["cycles"]) == cycles
    ms_step = elapsed * 1e3 / args.steps
    dfs_ms = float(np.mean([i["dfs_ms"] for i in infos]))
    hist_ms = float(np.mean([i["gpu_ms"] for i in infos]))

    W = 1 if int(sizes.max()) <= 64 else 2
    bpp = dfs_bytes_per_path(W)
    achieved = paths * bpp / (dfs_ms * 1e-3) / 1e9
    dt = elapsed / args.steps
    roofline = {"bound": "lds", "kernel": f"k_dfs<W={W}, count-only, batch>",
                "achieved": round(achieved, 1), "peak": round(LDS_PEAK_GBPS, 1),
                "unit": "GB/s", "frac": round(achieved / LDS_PEAK_GBPS, 4),
                "traffic": counted_traffic("k_dfs_batch4096.md"),
                "bytes_per_path": bpp, "paths_per_launch": paths,
                "avg_launch_us": round(dfs_ms * 1e3, 3),
                "measured": "HIP events around the depth-first launch on the batch's "
                            "stream, in every timed step"}
    roofline["depth_first_diag"] = _dfs_diag(infos[-1])
    if not baselines:
        return {"ms_per_step": round(ms_step, 4), "depth_first_ms": round(dfs_ms, 3),
                "value": round(cycles * args.steps / elapsed, 1), "roofline": roofline}

    # baseline A: the same kernels, one launch group per graph, same grid
    buf_a = np.zeros(total, np.int64)
    t0 = time.perf_counter()
    with cc.Batch(off_d, rp_d, ci_d, stream=stream, sizes=sizes, **opts) as h:
        h.histograms_into(buf_a, hoff, per_graph_launch=True)
        launches_a = h.last_run()["levels_launched"]
    torch.cuda.synchronize()
    dt_a = time.perf_counter() - t0
    check(buf_a, "per-graph launch")

    # baseline B: one cc_prepare + cc_histogram call per graph, each graph's
    # CSR resident on the device
    dev_graphs = [(g.n, torch.tensor(g.row_ptr, dtype=torch.int32, device="cuda"),
                   torch.tensor(g.col_idx if g.col_idx.size else np.zeros(1, np.int32),
                                dtype=torch.int32, device="cuda")) for g in b.graphs]
    buf_b = np.zeros(total, np.int64)

    def per_graph_calls(lo, hi):
        for g in range(lo, hi):
            n, rp, ci = dev_graphs[g]
            with cc.Graph(n, rp, ci, stream=stream) as h:
                buf_b[hoff[g]:hoff[g] + n + 1] = h.histogram()

    per_graph_calls(0, 64)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    per_graph_calls(0, G)
    torch.cuda.synchronize()
    dt_b = time.perf_counter() - t0
    check(buf_b, "per-graph calls")

    base = min(dt_a, dt_b)
    return {
        "ms_per_step": round(ms_step, 4),
        "value": round(cycles * args.steps / elapsed, 1),
        "config": {"workload": BATCH_WORKLOAD, "graphs": G, "cycles": cycles,
                   "paths_expanded": paths, "parallelism": "single GPU",
                   "launch": "persistent (stage one of every graph in one launch, one "
                             "persistent depth-first launch with work stealing)"},
        "paths_per_s": round(paths * args.steps / elapsed, 1),
        "roofline": roofline,
        "batched": {
            "parity": "every timed pass and both baselines equal the stored oracle histograms",
            "persistent": {"ms_per_pass": round(dt * 1e3, 3),
                           "histogram_call_gpu_ms": round(hist_ms, 3),
                           "depth_first_ms": round(dfs_ms, 3),
                           "cycles_per_s": round(cycles / dt, 1), "launches": 3},
            "per_graph_launch": {"ms": round(dt_a * 1e3, 3),
                                 "cycles_per_s": round(cycles / dt_a, 1),
                                 "launches": int(launches_a),
                                 "form": "prepare_batch, then stage one + depth-first launch "
                                         "per graph, the depth-first kernel on the same full "
                                         "grid as the persistent launch"},
            "per_graph_calls": {"ms": round(dt_b * 1e3, 3), "cycles_per_s": round(cycles / dt_b, 1),
                                "form": "cc_prepare + cc_histogram + cc_release per graph, each "
                                        "graph's CSR resident on the device"},
            "speedup": round(base / dt, 2),
            "speedup_vs": "per_graph_launch" if dt_a <= dt_b else "per_graph_calls",
            "autotuned": opts, "autotune_calibration_ms": tuned["ms"]},
    }


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
            "depth_first": {"ms": round(info["dfs_ms"], 4), **_dfs_diag(info),
                            "paths_per_s": round(
                                (paths - int(front[:info["switch_level"]].sum()))
                                / (info["dfs_ms"] * 1e-3), 1) if info["dfs_ms"] > 0 else 0.0},
            "stage1_ms": round(info["stage1_ms"], 4)}


def paging_section():
    """Grid 7x10 (8,136,453 cycles, 258M vertex ids): the whole output in one
    cc_enumerate call, against the same output paged through buffers of at
    most 64 Mi vertex ids (256 MiB), three ways: by ranges of stage-one roots
    out of one run grouped by root (cc_enumerate_by_roots), by ranges of
    roots with a run per page (cc_enumerate_roots; each page runs only the
    search below its roots), and by ranges of cycle lengths
    (cc_enumerate_lengths; each page reruns the whole enumeration).  The
    root pages are checked to add up to the histogram."""
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

        def by_lengths():
            pages = 0
            for _ in h.pages(max_verts=limit):
                pages += 1
            torch.cuda.synchronize()
            return pages

        def by_roots(check=False, one_run=None):
            pages, cyc, ids = 0, 0, 0
            for lo, hi, v, o in h.pages_by_roots(max_verts=limit, one_run=one_run):
                pages += 1
                if check:
                    cyc += o.numel() - 1
                    ids += int(o[-1])
            torch.cuda.synchronize()
            if check:
                assert cyc == nc and ids == nv
            return pages

        w = _timed(whole, warmup=2, runs=5)
        pages_l = by_lengths()
        pl = _timed(by_lengths, warmup=1, runs=3)
        pages_r = by_roots(check=True)
        pr = _timed(by_roots, warmup=1, runs=5)
        pages_rr = by_roots(check=True, one_run=False)
        prr = _timed(lambda: by_roots(one_run=False), warmup=1, runs=3)
    return {"workload": "grid 7x10, full enumeration", "cycles": nc, "vertex_ids": nv,
            "whole_ms": w, "page_limit_vertex_ids": limit,
            "by_roots": {"pages": pages_r, "ms": pr,
                         "vs_whole": round(pr["median"] / w["median"], 2),
                         "form": "one run grouped by root (cc_enumerate_by_roots), pages "
                                 "cut out of it (ids in place, offsets rebased)"},
            "by_roots_runs": {"pages": pages_rr, "ms": prr,
                              "vs_whole": round(prr["median"] / w["median"], 2),
                              "form": "one cc_enumerate_roots run per page"},
            "by_lengths": {"pages": pages_l, "ms": pl,
                           "vs_whole": round(pl["median"] / w["median"], 2)}}


def large_n_section():
    """Graphs of more than 128 vertices, full enumeration with CSR and
    results on the device: C_256, and 256 vertices made of two 6x8 grids,
    two 5x6 grids and C_100 with ids permuted (four-word bitsets); beyond
    256 vertices (sixteen words, rows in device memory) C_1024, 774 vertices
    made of four 6x8 and four 5x7 grids, C_300, a 100-spoke wheel, K_{4,5}
    and the 5-cube, and a random 1024-vertex tree with 20 extra edges."""
    import torch

    from paper_1410_4876_amd import cc
    from paper_1410_4876_amd import graphgen as gg

    union = gg.permute_random(gg.disjoint_union(gg.grid(6, 8), gg.grid(6, 8), gg.grid(5, 6),
                                                gg.grid(5, 6), gg.cycle(100)),
                              np.random.default_rng(256))
    union774 = gg.permute_random(
        gg.disjoint_union(*([gg.grid(6, 8)] * 4 + [gg.grid(5, 7)] * 4 +
                            [gg.cycle(300), gg.wheel(100), gg.complete_bipartite(4, 5),
                             gg.hypercube(5)])), np.random.default_rng(774))
    tree = gg.permute_random(gg.tree_plus_edges(1024, 20, np.random.default_rng(3)),
                             np.random.default_rng(33))
    out = []
    for g in [gg.cycle(256), union, gg.cycle(1024), union774, tree]:
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
    the serving loop; p50/p99 latency beside throughput.  Every reply is
    then checked against the same graph run alone (cc_prepare +
    cc_histogram)."""
    from paper_1410_4876_amd import cc, loadgen
    from paper_1410_4876_amd import graphgen as gg

    reqs = gg.request_stream(rate_hz=2000.0, duration_s=args.serve_seconds, k=5)
    with cc.Server() as sv:
        # warm-up: a short stream of its own, not part of the figures
        loadgen.run_stream(sv, gg.request_stream(rate_hz=2000.0, duration_s=0.2, k=1005))
        r = loadgen.run_stream(sv, reqs)
    out = {k: v for k, v in r.items() if k not in ("hists", "statuses")}
    t0 = time.perf_counter()
    bad = 0
    for q, h, st in zip(reqs, r["hists"], r["statuses"]):
        with cc.prepare(q.graph) as g:
            alone = g.histogram()
        if st != 0 or h is None or not np.array_equal(h, alone):
            bad += 1
    out["replies_equal_alone"] = bad == 0
    out["replies_checked"] = len(reqs)
    out["check_s"] = round(time.perf_counter() - t0, 1)
    assert bad == 0, f"{bad} serving replies differ from the graph run alone"
    out["workload"] = (f"Poisson stream at 2000 requests/s for {args.serve_seconds:g} s: "
                       "grids p x q (p, q in 3..7) and ER graphs (n in 20..80, d in [3,5]), "
                       "ids permuted")
    return out


def grid8x8_section(args):
    """8x8 grid (n=64, m=112, ids permuted), full enumeration as int32
    vertex lists into device buffers: whole passes (prepare, enumerate,
    release), the canonical cycle set's size checked against the stored
    oracle output, and the roofline of the breadth-first step kernel."""
    import torch

    from paper_1410_4876_amd import cc
    from paper_1410_4876_amd import graphgen as gg

    gold = json.load(open(GRID8X8))
    g = gg.workload_grid8x8()
    rp = torch.tensor(g.row_ptr, dtype=torch.int32, device="cuda")
    ci = torch.tensor(g.col_idx, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    n_cycles, n_verts = gold["total_cycles"], gold["total_verts"]
    verts = torch.empty(n_verts, dtype=torch.int32, device="cuda")
    offs = torch.empty(n_cycles + 1, dtype=torch.int64, device="cuda")

    def step(profile):
        with cc.Graph(g.n, rp, ci, stream=stream, profile=profile) as h:
            nc, nv = h.enumerate_into(verts, offs)
            assert nc == n_cycles and nv == n_verts
            return h.last_run(), h.frontier()

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = [step(False)[0] for _ in range(args.steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    info, front = step(False)
    assert front.tolist() == gold["front"]
    # a second pass with HIP events around every step launch
    pinfos = [step(True)[0] for _ in range(args.steps)]
    torch.cuda.synchronize()
    lvl_ms = sum(i["level_ms"] for i in pinfos)
    launches = sum(i["levels_launched"] for i in pinfos)
    avg_us = lvl_ms * 1e3 / max(launches, 1)
    model_bytes = sum(i["level_bytes"] for i in pinfos) / max(launches, 1)
    # the same figure with the survey's bytes per unit: 36 B per path
    # processed (X and S words and the end vertices, written once, read
    # once), per cycle 8 B of staged bitset and 4k + 8 B of output
    paths = int(info["paths"])
    W = 1
    per_step = paths * 2 * (16 * W + 2) + n_cycles * (8 * W + 8) + n_verts * 4
    unit_bytes = per_step / (launches / len(pinfos))
    ach_model = model_bytes / (avg_us * 1e-6) / 1e9
    ach_unit = unit_bytes / (avg_us * 1e-6) / 1e9
    return {"workload": "grid 8x8 (n=64, m=112), ids permuted, full enumeration to int32 "
                        "vertex lists", "cycles": n_cycles, "vertices_out": n_verts,
            "paths_expanded": paths, "ms_per_step": round(elapsed * 1e3 / args.steps, 4),
            "cycles_per_s": round(n_cycles * args.steps / elapsed, 1),
            "paths_per_s": round(paths * args.steps / elapsed, 1),
            "roofline": {"bound": "hbm", "kernel": "k_step (breadth-first step: one or two "
                                                  "levels per launch, staged-cycle decode)",
                         "achieved": round(ach_unit, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                         "frac": round(ach_unit / HBM_PEAK_GBPS, 4),
                         "bytes_per_launch": round(unit_bytes, 1),
                         "bytes_rule": "36 B per path processed + (8W + 8) B per cycle + 4 B "
                                       "per output vertex id, over the step launches",
                         "model_bytes_per_launch": round(model_bytes, 1),
                         "model_achieved": round(ach_model, 1),
                         "model_frac": round(ach_model / HBM_PEAK_GBPS, 4),
                         "traffic": counted_traffic("k_step_grid8x8_enumerate.md"),
                         "avg_launch_us": round(avg_us, 3),
                         "launches_per_step": round(launches / len(pinfos), 1),
                         "measured": "HIP events around every step launch, second pass of "
                                     "the timed steps"},
            "breakdown_ms": {
                "stage1": round(sum(i["stage1_ms"] for i in pinfos) / len(pinfos), 4),
                "head": round(sum(i["head_ms"] for i in pinfos) / len(pinfos), 4),
                "levels": round(lvl_ms / len(pinfos), 4),
                "dfs": round(sum(i["dfs_ms"] for i in pinfos) / len(pinfos), 4)},
            "head_steps": pinfos[-1]["head_steps"]}


SECTIONS = ["batched", "batched_persistent", "grid8x8", "er40", "grid7x12", "paging", "large_n", "table1",
            "serving", "cpu"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="time budget of each bounded oracle sample")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only time a plain 1 GiB device-to-device copy (counter calibration)")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="length of the replayed request stream")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving stream")
    ap.add_argument("--no-table1", action="store_true",
                    help="skip the structured graphs of the paper's Table 1")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the 8x8, ER G(40,100), 7x12, paging and large-graph sections")
    ap.add_argument("--section", choices=SECTIONS,
                    help="run only this section and print its JSON (for profiling one workload)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; the path shards by triplet "
                                   "or by graph across GPUs, which is not built here",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    # the oracle runs first, on forked workers, before this process touches the GPU
    cpu = None
    if args.section == "cpu" or (not args.section and not args.no_cpu_baseline):
        cpu = cpu_baselines(args.cpu_seconds)
        if args.section == "cpu":
            print(json.dumps({"cpu": cpu}), flush=True)
            return

    import torch

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        # A plain copy of known size: what the HBM byte counters read for it
        # scales the counters read for the kernels.
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
    if args.section:
        fn = {"er40": er40_section, "grid7x12": grid7x12_section, "paging": paging_section,
              "large_n": large_n_section, "grid8x8": lambda: grid8x8_section(args),
              "table1": lambda: table1_section(args), "batched": lambda: batched_headline(args),
              "batched_persistent": lambda: batched_headline(args, baselines=False),
              "serving": lambda: serving_section(args)}[args.section]
        print(json.dumps({args.section: fn()}), flush=True)
        return

    head = batched_headline(args)
    out = {
        "metric": "chordless cycles/s on 1 MI355X, batched vs per-graph launch; p99 latency",
        "value": head["value"],
        "unit": "chordless cycles/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64", "data": "synthetic",
        "config": head["config"],
        "paths_per_s": head["paths_per_s"],
        "roofline": head["roofline"],
        "batched": head["batched"],
    }
    print(json.dumps({"progress": "batched", "value": out["value"],
                      "speedup": out["batched"]["speedup"]}), file=sys.stderr, flush=True)
    if not args.no_serve:
        out["serving"] = serving_section(args)
        out["p99_latency_ms"] = out["serving"]["latency_ms"]["p99"]
        print(json.dumps({"progress": "serving", "latency_ms": out["serving"]["latency_ms"]}),
              file=sys.stderr, flush=True)
    if not args.no_extra:
        out["grid8x8"] = grid8x8_section(args)
        out["er40"] = er40_section()
        out["grid7x12"] = grid7x12_section()
        out["paging"] = paging_section()
        out["large_n"] = large_n_section()
        print(json.dumps({"progress": "sections"}), file=sys.stderr, flush=True)
    if not args.no_table1:
        out["table1"] = table1_section(args)
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
