"""Autotuner for the depth-first engine's launch parameters.

The persistent depth-first kernel has three knobs: wavefronts per CU, the
number of paths a wavefront must hold before it answers a work request, and
how many handed-over paths a wavefront claims per atomic.  tune_batch()
times every candidate on a held-out calibration batch (a different seed from
any workload it is used on), keeps the fastest, and caches the choice as
JSON keyed by the device name, the workload class, the candidate grid and a
hash of the library's sources (a choice made for other kernels is not
reused).
"""
from __future__ import annotations

import itertools
import json
import os
import time

import numpy as np

DEFAULT_GRID = {
    "dfs_waves_per_cu": [8, 12, 16, 24, 32],
    "dfs_donate_min": [64, 128, 256],
    "dfs_claim": [0, 128, 1024],
}


def _cache_path() -> str:
    base = os.environ.get("CC_AUTOTUNE_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "cc_autotune.json")
    return base


def _device_key() -> str:
    import torch
    p = torch.cuda.get_device_properties(0)
    return f"{getattr(p, 'gcnArchName', p.name)}:{p.multi_processor_count}cu"


def _load_cache(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def tune_batch(workload_class: str = "er_n16-64_d2.5-5", calibration=None, grid=None,
               repeats: int = 2, force: bool = False, cache_path: str | None = None) -> dict:
    """Best options for batched runs of `workload_class`.  `calibration` is a
    graphgen.Batch (default: 4096 ER graphs shaped like the 4096-graph
    workload, seed index 1004; a smaller calibration batch has too little
    work per wavefront and favours too few wavefronts).  Returns {"options": {...}, "ms": best,
    "table": [...]}."""
    from . import cc
    from . import graphgen as gg

    from .build import sources_sha256

    cache_path = cache_path or _cache_path()
    grid = grid or DEFAULT_GRID
    grid_key = json.dumps(grid, sort_keys=True)
    key = f"{_device_key()}|{workload_class}|cal4096|{grid_key}|{sources_sha256()[:16]}"
    cache = _load_cache(cache_path)
    if key in cache and not force:
        return cache[key]
    if calibration is None:
        calibration = gg.pack_batch(gg.er_batch_graphs(4096, k=1004))
    names = list(grid)
    table = []
    ref = None
    for values in itertools.product(*(grid[k] for k in names)):
        opts = dict(zip(names, values))
        with cc.prepare_batch(calibration, **opts) as h:
            out = h.histograms()  # warm-up, and the result every candidate must match
            if ref is None:
                ref = out
            elif not np.array_equal(out, ref):
                raise RuntimeError(f"autotune: candidate {opts} changed the result")
            best = float("inf")
            for _ in range(repeats):
                t = time.perf_counter()
                h.histograms()
                best = min(best, time.perf_counter() - t)
        table.append({"options": opts, "ms": round(best * 1e3, 4)})
    table.sort(key=lambda r: r["ms"])
    result = {"options": table[0]["options"], "ms": table[0]["ms"], "table": table,
              "calibration_graphs": len(calibration.graphs)}
    cache[key] = result
    try:
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    except OSError:
        pass
    return result
