"""CPU oracle for chordless-cycle enumeration -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product path (the HIP library and its binding)
never imports, links or runs anything here, and this package imports
nothing from the product package.

The arithmetic lives in ``cc_oracle.c`` (plain C, compiled with gcc): the
paper's Algorithm 1 in depth-first form with sorted adjacency lists and
binary-search adjacency tests.  This module only marshals arguments.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import sys
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cc_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

OK, ERR_INVALID_ARG, ERR_NOT_SIMPLE, ERR_OUT_OF_MEMORY, ERR_INTERNAL = 0, -1, -2, -5, -7
INT64_MAX = (1 << 63) - 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no GPU code involved)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-shared",
                               "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            lib = ctypes.CDLL(_LIB)
            i32p = ctypes.POINTER(ctypes.c_int32)
            i64p = ctypes.POINTER(ctypes.c_int64)
            lib.orc_validate.argtypes = [ctypes.c_int32, i32p, i32p]
            lib.orc_validate.restype = ctypes.c_int
            lib.orc_degree_labelling.argtypes = [ctypes.c_int32, i32p, i32p, i32p]
            lib.orc_degree_labelling.restype = ctypes.c_int
            lib.orc_count_roots.argtypes = [ctypes.c_int32, i32p, i32p]
            lib.orc_count_roots.restype = ctypes.c_int64
            lib.orc_enumerate.argtypes = [ctypes.c_int32, i32p, i32p, ctypes.c_int64,
                                          ctypes.c_int64, i64p, i64p, i32p, i32p,
                                          ctypes.c_int64, i64p, ctypes.c_int64, i64p, i64p]
            lib.orc_enumerate.restype = ctypes.c_int
            _lib = lib
    return _lib


def _p32(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _p64(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _arrays(row_ptr, col_idx):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    if ci.size == 0:
        ci = np.zeros(1, np.int32)
    return rp, ci


def validate(n, row_ptr, col_idx) -> int:
    rp, ci = _arrays(row_ptr, col_idx)
    return _load().orc_validate(n, _p32(rp), _p32(ci))


def degree_labelling(n, row_ptr, col_idx) -> np.ndarray:
    rp, ci = _arrays(row_ptr, col_idx)
    lab = np.zeros(max(n, 1), np.int32)
    st = _load().orc_degree_labelling(n, _p32(rp), _p32(ci), _p32(lab))
    if st != OK:
        raise ValueError(f"oracle: invalid graph ({st})")
    return lab[:n]


def count_roots(n, row_ptr, col_idx) -> int:
    rp, ci = _arrays(row_ptr, col_idx)
    c = _load().orc_count_roots(n, _p32(rp), _p32(ci))
    if c < 0:
        raise ValueError(f"oracle: invalid graph ({c})")
    return int(c)


class Result:
    """hist[k]: cycles with k vertices; front[t]: paths with t vertices
    expanded; labels; cycles: list of int32 arrays in path order (or None)."""

    def __init__(self, hist, front, labels, cycles, n_cycles, n_verts):
        self.hist = hist
        self.front = front
        self.labels = labels
        self.cycles = cycles
        self.n_cycles = n_cycles
        self.n_verts = n_verts

    @property
    def count(self) -> int:
        return int(self.hist.sum())


def enumerate_cycles(n, row_ptr, col_idx, want_cycles=True, root_lo=0, root_hi=INT64_MAX,
                     max_verts=None) -> Result:
    """Run the oracle.  With want_cycles the cycles are stored (two passes:
    a counting pass sizes the buffers, then the storing pass)."""
    lib = _load()
    rp, ci = _arrays(row_ptr, col_idx)
    hist = np.zeros(n + 1, np.int64)
    front = np.zeros(n + 1, np.int64)
    lab = np.zeros(max(n, 1), np.int32)
    nc = ctypes.c_int64(0)
    nv = ctypes.c_int64(0)
    st = lib.orc_enumerate(n, _p32(rp), _p32(ci), root_lo, root_hi, _p64(hist), _p64(front),
                           _p32(lab), None, 0, None, 0, ctypes.byref(nc), ctypes.byref(nv))
    if st != OK:
        raise ValueError(f"oracle: status {st}")
    cycles = None
    if want_cycles:
        if max_verts is not None and nv.value > max_verts:
            raise MemoryError("oracle: cycle output larger than max_verts")
        verts = np.zeros(max(nv.value, 1), np.int32)
        offs = np.zeros(nc.value + 1, np.int64)
        h2 = np.zeros(n + 1, np.int64)
        f2 = np.zeros(n + 1, np.int64)
        nc2 = ctypes.c_int64(0)
        nv2 = ctypes.c_int64(0)
        st = lib.orc_enumerate(n, _p32(rp), _p32(ci), root_lo, root_hi, _p64(h2), _p64(f2),
                               None, _p32(verts), nv.value, _p64(offs), nc.value,
                               ctypes.byref(nc2), ctypes.byref(nv2))
        if st != OK or nc2.value != nc.value:
            raise ValueError("oracle: second pass disagrees")
        cycles = (verts, offs)
    return Result(hist, front, lab[:n], cycles, nc.value, nv.value)


def enumerate_single_pass(n, row_ptr, col_idx, verts_cap, cyc_cap, root_lo=0,
                          root_hi=INT64_MAX) -> Result:
    """One oracle pass that counts and stores the cycles into buffers of the
    given capacities (cycles beyond them are counted, not stored)."""
    lib = _load()
    rp, ci = _arrays(row_ptr, col_idx)
    hist = np.zeros(n + 1, np.int64)
    front = np.zeros(n + 1, np.int64)
    lab = np.zeros(max(n, 1), np.int32)
    verts = np.zeros(max(int(verts_cap), 1), np.int32)
    offs = np.zeros(int(cyc_cap) + 1, np.int64)
    nc = ctypes.c_int64(0)
    nv = ctypes.c_int64(0)
    st = lib.orc_enumerate(n, _p32(rp), _p32(ci), root_lo, root_hi, _p64(hist), _p64(front),
                           _p32(lab), _p32(verts), int(verts_cap), _p64(offs), int(cyc_cap),
                           ctypes.byref(nc), ctypes.byref(nv))
    if st != OK:
        raise ValueError(f"oracle: status {st}")
    return Result(hist, front, lab[:n], (verts, offs), nc.value, nv.value)


def cycle_list(res: Result):
    """The stored cycles as a list of int32 arrays (path order)."""
    verts, offs = res.cycles
    return [verts[offs[i]:offs[i + 1]] for i in range(len(offs) - 1)]


def _worker(args):
    n, rp, ci, lo, hi = args
    r = enumerate_cycles(n, rp, ci, want_cycles=False, root_lo=lo, root_hi=hi)
    return r.hist, r.front


def histogram_parallel(n, row_ptr, col_idx, procs=None, splits=None):
    """Histogram and frontier counts with the roots split over processes
    (each process runs the same sequential oracle on a range of roots)."""
    import multiprocessing as mp
    roots = count_roots(n, row_ptr, col_idx)
    procs = procs or os.cpu_count() or 1
    splits = splits or max(1, min(roots, procs * 8))
    bounds = np.linspace(0, roots, splits + 1).astype(np.int64)
    jobs = [(n, np.asarray(row_ptr), np.asarray(col_idx), int(bounds[i]), int(bounds[i + 1]))
            for i in range(splits)]
    hist = np.zeros(n + 1, np.int64)
    front = np.zeros(n + 1, np.int64)
    ctx = mp.get_context("fork" if sys.platform.startswith("linux") else "spawn")
    with ctx.Pool(procs) as pool:
        for h, f in pool.imap_unordered(_worker, jobs):
            hist += h
            front += f
    return hist, front
