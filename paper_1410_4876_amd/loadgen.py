"""Open-loop load generator for the serving loop.

Replays a request stream (graphgen.request_stream: Poisson arrivals) against
a cc.Server on the stream's own clock: requests are submitted at their
arrival times whether or not earlier ones have finished, and a collector
thread takes the replies.  Latency is the server's own submit-to-completion
time.  Reports p50/p99 latency beside throughput.
"""
from __future__ import annotations

import threading
import time

import numpy as np


def run_stream(server, requests, result_timeout_s: float = 300.0) -> dict:
    """Submit `requests` (objects with .arrival_s and .graph) to `server` on
    their arrival clock; wait for every reply.  Returns latency percentiles,
    throughput and per-request histograms."""
    ids = []
    hists = [None] * len(requests)
    lats = np.zeros(len(requests))
    statuses = np.zeros(len(requests), np.int32)
    ready = threading.Condition()
    errors = []

    def collect():
        i = 0
        while i < len(requests):
            with ready:
                while len(ids) <= i:
                    ready.wait()
                rid = ids[i]
            try:
                h, lat, st = server.result(rid, timeout_s=result_timeout_s)
            except Exception as e:  # keep draining, report at the end
                errors.append(e)
                h, lat, st = None, float("nan"), -1
            hists[i] = h
            lats[i] = lat
            statuses[i] = st
            i += 1

    th = threading.Thread(target=collect, daemon=True)
    th.start()
    late = 0.0
    t0 = time.perf_counter()
    for r in requests:
        delay = r.arrival_s - (time.perf_counter() - t0)
        if delay > 0:
            time.sleep(delay)
        else:
            late = max(late, -delay)
        rid = server.submit_graph(r.graph)
        with ready:
            ids.append(rid)
            ready.notify()
    t_submitted = time.perf_counter() - t0
    th.join()
    wall = time.perf_counter() - t0
    if errors:
        raise errors[0]
    ok = statuses == 0
    cycles = int(sum(int(h.sum()) for h, s in zip(hists, ok) if s))
    offered = len(requests) / max(requests[-1].arrival_s, 1e-9) if requests else 0.0
    return {
        "requests": len(requests),
        "ok": int(ok.sum()),
        "offered_rate_hz": round(offered, 1),
        "achieved_rate_hz": round(len(requests) / wall, 1),
        "wall_s": round(wall, 3),
        "submit_s": round(t_submitted, 3),
        "max_submit_lag_ms": round(late * 1e3, 3),
        "cycles": cycles,
        "cycles_per_s": round(cycles / wall, 1),
        "latency_ms": {
            "p50": round(float(np.percentile(lats, 50)), 3),
            "p90": round(float(np.percentile(lats, 90)), 3),
            "p99": round(float(np.percentile(lats, 99)), 3),
            "max": round(float(lats.max()), 3),
            "mean": round(float(lats.mean()), 3),
        },
        "stats": server.stats(),
        "hists": hists,
        "statuses": statuses,
    }
