"""Python binding of libcc (argument marshalling only).

Every computation runs in the HIP kernels behind the C ABI declared in
include/cc.h; this module converts numpy arrays / torch tensors into
pointers, sizes and a HIP stream, and raises on error statuses.  There is no
CPU fallback: if libcc.so is missing or no gfx950 device is present, calls
fail loudly.
"""
from __future__ import annotations

import ctypes
import os
import sys
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcc.so")

CC_OK = 0
CC_ERR_INVALID_ARG = -1
CC_ERR_NOT_SIMPLE = -2
CC_ERR_TOO_LARGE = -3
CC_ERR_BUFFER_TOO_SMALL = -4
CC_ERR_OUT_OF_MEMORY = -5
CC_ERR_DEVICE = -6
CC_ERR_NO_DEVICE = -7
CC_ERR_NOT_READY = -8
CC_ERR_INTERNAL = -9

CC_INPUT_DEVICE = 1 << 0
CC_OUTPUT_DEVICE = 1 << 1
CC_FORCE_DFS = 1 << 2
CC_PROFILE = 1 << 3
CC_ONE_LEVEL_STEPS = 1 << 5
CC_SORTED = 1 << 6
CC_MAX_VERTICES = 1024
CC_MAX_BATCH_VERTICES = 256
CC_BATCH_PERSISTENT = 0
CC_BATCH_PER_GRAPH = 1

_lock = threading.Lock()
_lib = None


class CCError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} ({status})")


class Options(ctypes.Structure):
    _fields_ = [("stream", ctypes.c_void_p),
                ("frontier_budget_bytes", ctypes.c_int64),
                ("flags", ctypes.c_uint32),
                ("dfs_level", ctypes.c_int32),
                ("dfs_waves_per_cu", ctypes.c_int32),
                ("bfs_blocks", ctypes.c_int32),
                ("dfs_donate_min", ctypes.c_int32),
                ("dfs_claim", ctypes.c_int32)]


class RunInfo(ctypes.Structure):
    _fields_ = [("cycles", ctypes.c_int64),
                ("paths", ctypes.c_int64),
                ("peak_frontier", ctypes.c_int64),
                ("switch_level", ctypes.c_int32),
                ("levels_launched", ctypes.c_int32),
                ("gpu_ms", ctypes.c_double),
                ("stage1_ms", ctypes.c_double),
                ("level_ms", ctypes.c_double),
                ("dfs_ms", ctypes.c_double),
                ("level_bytes", ctypes.c_int64),
                ("device_diag", ctypes.c_int64),
                ("head_steps", ctypes.c_int32),
                ("reserved", ctypes.c_int32),
                ("head_ms", ctypes.c_double),
                ("head_bytes", ctypes.c_int64),
                ("dfs_steps", ctypes.c_int64),
                ("dfs_donations", ctypes.c_int64),
                ("dfs_lane_use", ctypes.c_double),
                ("dfs_idle_frac", ctypes.c_double),
                ("dfs_fills", ctypes.c_int64),
                ("dfs_spills", ctypes.c_int64),
                ("dfs_global_adds", ctypes.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class ServerOptions(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int32), ("max_batch_graphs", ctypes.c_int32),
                ("slot_root_slots", ctypes.c_int64), ("slot_work_bytes", ctypes.c_int64),
                ("dfs_waves_per_cu", ctypes.c_int32), ("reserved", ctypes.c_int32)]


def lib():
    """Load libcc.so (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError(f"libcc.so not built ({LIB_PATH}); run __graft_entry__.build()")
            L = ctypes.CDLL(LIB_PATH)
            vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
            pp = ctypes.POINTER(ctypes.c_void_p)
            L.cc_prepare.argtypes = [i32, vp, vp, ctypes.POINTER(Options), pp]
            L.cc_prepare.restype = ctypes.c_int
            L.cc_count.argtypes = [vp, ctypes.POINTER(i64)]
            L.cc_count.restype = ctypes.c_int
            L.cc_histogram.argtypes = [vp, vp, i32]
            L.cc_histogram.restype = ctypes.c_int
            L.cc_enumerate.argtypes = [vp, vp, i64, vp, i64, ctypes.POINTER(i64), ctypes.POINTER(i64)]
            L.cc_enumerate.restype = ctypes.c_int
            L.cc_enumerate_lengths.argtypes = [vp, i32, i32, vp, i64, vp, i64,
                                               ctypes.POINTER(i64), ctypes.POINTER(i64)]
            L.cc_enumerate_lengths.restype = ctypes.c_int
            L.cc_root_total.argtypes = [vp, ctypes.POINTER(i64)]
            L.cc_root_total.restype = ctypes.c_int
            L.cc_histogram_roots.argtypes = [vp, i64, i64, vp, i32]
            L.cc_histogram_roots.restype = ctypes.c_int
            L.cc_enumerate_roots.argtypes = [vp, i64, i64, vp, i64, vp, i64,
                                             ctypes.POINTER(i64), ctypes.POINTER(i64)]
            L.cc_enumerate_roots.restype = ctypes.c_int
            L.cc_enumerate_by_roots.argtypes = [vp, vp, i64, vp, i64, vp, i64,
                                                ctypes.POINTER(i64), ctypes.POINTER(i64)]
            L.cc_enumerate_by_roots.restype = ctypes.c_int
            L.cc_labels.argtypes = [vp, vp]
            L.cc_labels.restype = ctypes.c_int
            L.cc_frontier.argtypes = [vp, vp, i32]
            L.cc_frontier.restype = ctypes.c_int
            L.cc_level_times.argtypes = [vp, vp, i32]
            L.cc_level_times.restype = ctypes.c_int
            L.cc_last_run.argtypes = [vp, ctypes.POINTER(RunInfo)]
            L.cc_last_run.restype = ctypes.c_int
            L.cc_release.argtypes = [vp]
            L.cc_release.restype = None
            L.cc_status_string.argtypes = [ctypes.c_int]
            L.cc_status_string.restype = ctypes.c_char_p
            L.cc_abi_version.argtypes = []
            L.cc_abi_version.restype = i32
            L.cc_prepare_batch.argtypes = [i32, vp, vp, vp, ctypes.POINTER(Options), pp]
            L.cc_prepare_batch.restype = ctypes.c_int
            L.cc_histogram_batch.argtypes = [vp, vp, vp]
            L.cc_histogram_batch.restype = ctypes.c_int
            L.cc_histogram_batch_mode.argtypes = [vp, vp, vp, i32]
            L.cc_histogram_batch_mode.restype = ctypes.c_int
            L.cc_batch_labels.argtypes = [vp, vp]
            L.cc_batch_labels.restype = ctypes.c_int
            L.cc_batch_last_run.argtypes = [vp, ctypes.POINTER(RunInfo)]
            L.cc_batch_last_run.restype = ctypes.c_int
            L.cc_release_batch.argtypes = [vp]
            L.cc_release_batch.restype = None
            L.cc_server_create.argtypes = [ctypes.POINTER(ServerOptions), pp]
            L.cc_server_create.restype = ctypes.c_int
            L.cc_server_submit.argtypes = [vp, i32, vp, vp, ctypes.POINTER(i64)]
            L.cc_server_submit.restype = ctypes.c_int
            L.cc_server_result.argtypes = [vp, i64, ctypes.c_double, vp, i32,
                                           ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_int)]
            L.cc_server_result.restype = ctypes.c_int
            L.cc_server_stats.argtypes = [vp, vp, i32]
            L.cc_server_stats.restype = ctypes.c_int
            L.cc_server_destroy.argtypes = [vp]
            L.cc_server_destroy.restype = None
            _lib = L
    return _lib


def status_string(status: int) -> str:
    return lib().cc_status_string(status).decode()


def _check(st: int, where: str, info_fn=None):
    if st != CC_OK:
        err = CCError(st, where)
        if st == CC_ERR_INTERNAL and info_fn is not None:
            # which device-side check failed: kind << 24 | low bits of the value
            info = RunInfo()
            if info_fn(ctypes.byref(info)) == CC_OK:
                err.device_diag = int(info.device_diag)
                err.args = (f"{err.args[0]} [device_diag 0x{err.device_diag:08x}]",)
        raise err


_torch_types: dict = {}


def _is_torch(x) -> bool:
    t = type(x)
    r = _torch_types.get(t)
    if r is None:
        r = _torch_types[t] = t.__module__.startswith("torch")
    return r


def _ptr(x):
    """(pointer, is_device, keepalive) for a numpy array or torch tensor."""
    if x is None:
        return None, False, None
    if _is_torch(x):
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return ctypes.c_void_p(x.data_ptr()), bool(x.is_cuda), x
    a = np.ascontiguousarray(x)
    return ctypes.c_void_p(a.ctypes.data), False, a


def _stream_handle(stream) -> int | None:
    """A hipStream_t for the library: the given stream (torch.cuda.Stream or
    a raw handle), else torch's current stream once torch has set up the GPU
    (so device tensors written on a side stream are ordered before the
    library's work), else the null stream."""
    if stream is None:
        torch = sys.modules.get("torch")
        if torch is not None and torch.cuda.is_initialized():
            return int(torch.cuda.current_stream().cuda_stream)
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


class Graph:
    """A prepared graph (cc_prepare).  Use as a context manager or call
    release()."""

    def __init__(self, n, row_ptr, col_idx, stream=None, budget_bytes: int = 0,
                 force_dfs_level: int | None = None, dfs_waves_per_cu: int = 0,
                 bfs_blocks: int = 0, output_device: bool = True, profile: bool = False,
                 dfs_donate_min: int = 0, dfs_claim: int = 0, one_level_steps: bool = False,
                 sorted_output: bool = False):
        L = lib()
        rp, rp_dev, self._k1 = _ptr(_as_i32(row_ptr))
        ci, ci_dev, self._k2 = _ptr(_as_i32(col_idx))
        if rp_dev != ci_dev and n > 0:
            raise ValueError("row_ptr and col_idx must both be host or both be device")
        flags = 0
        if rp_dev:
            flags |= CC_INPUT_DEVICE
        if output_device:
            flags |= CC_OUTPUT_DEVICE
        if force_dfs_level is not None:
            flags |= CC_FORCE_DFS
        if profile:
            flags |= CC_PROFILE
        if one_level_steps:
            flags |= CC_ONE_LEVEL_STEPS
        if sorted_output:
            flags |= CC_SORTED
        self.opt = Options(_stream_handle(stream), int(budget_bytes), flags,
                           int(force_dfs_level or 0), int(dfs_waves_per_cu), int(bfs_blocks),
                           int(dfs_donate_min), int(dfs_claim))
        self.n = int(n)
        self.output_device = output_device
        h = ctypes.c_void_p()
        st = L.cc_prepare(self.n, rp, ci, ctypes.byref(self.opt), ctypes.byref(h))
        self._k1 = self._k2 = None
        _check(st, "cc_prepare")
        self.h = h

    # -- lifetime
    def release(self):
        if getattr(self, "h", None):
            lib().cc_release(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.release()

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass

    def _info_fn(self, p):
        return lib().cc_last_run(self.h, p)

    # -- calls
    def count(self) -> int:
        total = ctypes.c_int64()
        _check(lib().cc_count(self.h, ctypes.byref(total)), "cc_count", self._info_fn)
        return total.value

    def histogram(self) -> np.ndarray:
        h = np.zeros(self.n + 1, np.int64)
        _check(lib().cc_histogram(self.h, ctypes.c_void_p(h.ctypes.data), h.size), "cc_histogram",
               self._info_fn)
        self._hist = h.copy()
        return h

    def _sizes(self) -> np.ndarray:
        """The histogram, from an earlier call when there was one (it only
        depends on the graph)."""
        h = getattr(self, "_hist", None)
        return h.copy() if h is not None else self.histogram()

    def enumerate_into(self, verts, offsets):
        """Fill caller buffers (torch device tensors when the graph was
        prepared with output_device=True, else numpy arrays).  Returns
        (n_cycles, n_verts); raises CCError(CC_ERR_BUFFER_TOO_SMALL) with
        .required = (n_cycles, n_verts) if they do not fit."""
        vp, _, _ = _ptr(verts)
        op, _, _ = _ptr(offsets)
        nc, nv = ctypes.c_int64(), ctypes.c_int64()
        vcap = int(verts.numel() if _is_torch(verts) else np.asarray(verts).size)
        ccap = int(offsets.numel() if _is_torch(offsets) else np.asarray(offsets).size) - 1
        st = lib().cc_enumerate(self.h, vp, vcap, op, max(ccap, 0), ctypes.byref(nc), ctypes.byref(nv))
        if st == CC_ERR_INTERNAL:
            _check(st, "cc_enumerate", self._info_fn)
        if st != CC_OK:
            err = CCError(st, "cc_enumerate")
            err.required = (nc.value, nv.value)
            raise err
        return nc.value, nv.value

    def enumerate(self, device="cuda"):
        """Size exactly (histogram), allocate, enumerate.  Returns
        (verts, offsets) as torch tensors on `device` when prepared with
        output_device=True, else numpy arrays."""
        h = self.histogram()
        nc = int(h.sum())
        nv = int((h * np.arange(h.size)).sum())
        if self.output_device:
            import torch
            verts = torch.empty(max(nv, 1), dtype=torch.int32, device=device)
            offs = torch.empty(nc + 1, dtype=torch.int64, device=device)
        else:
            verts = np.empty(max(nv, 1), np.int32)
            offs = np.empty(nc + 1, np.int64)
        got_c, got_v = self.enumerate_into(verts, offs)
        assert got_c == nc and got_v == nv
        return verts[:nv], offs

    def enumerate_lengths_into(self, k_min: int, k_max: int, verts, offsets):
        """Fill caller buffers with the cycles of k_min..k_max vertices only
        (cc_enumerate_lengths).  Returns (n_cycles, n_verts); raises
        CCError(CC_ERR_BUFFER_TOO_SMALL) with .required if they do not fit."""
        vp, _, _ = _ptr(verts)
        op, _, _ = _ptr(offsets)
        nc, nv = ctypes.c_int64(), ctypes.c_int64()
        vcap = int(verts.numel() if _is_torch(verts) else np.asarray(verts).size)
        ccap = int(offsets.numel() if _is_torch(offsets) else np.asarray(offsets).size) - 1
        st = lib().cc_enumerate_lengths(self.h, int(k_min), int(k_max), vp, vcap, op,
                                        max(ccap, 0), ctypes.byref(nc), ctypes.byref(nv))
        if st == CC_ERR_INTERNAL:
            _check(st, "cc_enumerate_lengths", self._info_fn)
        if st != CC_OK:
            err = CCError(st, "cc_enumerate_lengths")
            err.required = (nc.value, nv.value)
            raise err
        return nc.value, nv.value

    def enumerate_lengths(self, k_min: int, k_max: int, device="cuda"):
        """The cycles of k_min..k_max vertices, sized exactly from the
        histogram: (verts, offsets) as torch tensors (output_device=True)
        or numpy arrays."""
        h = self._sizes()
        k = np.arange(h.size)
        sel = (k >= k_min) & (k <= k_max)
        nc = int(h[sel].sum())
        nv = int((h[sel] * k[sel]).sum())
        if self.output_device:
            import torch
            verts = torch.empty(max(nv, 1), dtype=torch.int32, device=device)
            offs = torch.empty(nc + 1, dtype=torch.int64, device=device)
        else:
            verts = np.empty(max(nv, 1), np.int32)
            offs = np.empty(nc + 1, np.int64)
        got_c, got_v = self.enumerate_lengths_into(k_min, k_max, verts, offs)
        assert got_c == nc and got_v == nv
        return verts[:nv], offs

    def pages(self, max_verts: int, max_cycles: int | None = None, device="cuda"):
        """Yield (k_min, k_max, verts, offsets) over consecutive ranges of
        cycle lengths, each holding at most max_verts vertex ids (and
        max_cycles cycles): the whole output in pieces that fit a bounded
        buffer.  Raises ValueError if a single length does not fit."""
        h = self._sizes()
        lens = [k for k in range(h.size) if h[k]]
        i = 0
        while i < len(lens):
            k0 = lens[i]
            nv = nc = 0
            j = i
            while j < len(lens):
                k = lens[j]
                v2, c2 = nv + int(h[k]) * k, nc + int(h[k])
                if v2 > max_verts or (max_cycles is not None and c2 > max_cycles):
                    break
                nv, nc = v2, c2
                j += 1
            if j == i:
                raise ValueError(f"the {int(h[k0])} cycles of length {k0} need "
                                 f"{int(h[k0]) * k0} vertex ids, more than max_verts={max_verts}")
            k1 = lens[j - 1]
            v, o = self.enumerate_lengths(k0, k1, device=device)
            yield k0, k1, v, o
            i = j

    # -- pages by ranges of stage-one roots
    def root_total(self) -> int:
        """Number of stage-one roots (cc_root_total)."""
        r = ctypes.c_int64()
        _check(lib().cc_root_total(self.h, ctypes.byref(r)), "cc_root_total")
        return r.value

    def histogram_roots(self, root_lo: int, root_hi: int) -> np.ndarray:
        """Histogram of the cycles found from roots root_lo..root_hi-1."""
        h = np.zeros(self.n + 1, np.int64)
        _check(lib().cc_histogram_roots(self.h, int(root_lo), int(root_hi),
                                        ctypes.c_void_p(h.ctypes.data), h.size),
               "cc_histogram_roots", self._info_fn)
        return h

    def enumerate_roots_into(self, root_lo: int, root_hi: int, verts, offsets):
        """The cycles found from roots root_lo..root_hi-1 into caller buffers.
        Returns (n_cycles, n_verts); raises CCError(CC_ERR_BUFFER_TOO_SMALL)
        with .required if they do not fit."""
        vp, _, _ = _ptr(verts)
        op, _, _ = _ptr(offsets)
        nc, nv = ctypes.c_int64(), ctypes.c_int64()
        vcap = int(verts.numel() if _is_torch(verts) else np.asarray(verts).size)
        ccap = int(offsets.numel() if _is_torch(offsets) else np.asarray(offsets).size) - 1
        st = lib().cc_enumerate_roots(self.h, int(root_lo), int(root_hi), vp, vcap, op,
                                      max(ccap, 0), ctypes.byref(nc), ctypes.byref(nv))
        if st == CC_ERR_INTERNAL:
            _check(st, "cc_enumerate_roots", self._info_fn)
        if st != CC_OK:
            err = CCError(st, "cc_enumerate_roots")
            err.required = (nc.value, nv.value)
            raise err
        return nc.value, nv.value

    def enumerate_by_roots_into(self, verts, offsets, root_first):
        """The whole output grouped by stage-one root (cc_enumerate_by_roots)
        into caller buffers; root_first holds root_total() + 1 entries.
        Returns (n_cycles, n_verts); raises CCError(CC_ERR_BUFFER_TOO_SMALL)
        with .required if they do not fit."""
        vp, _, _ = _ptr(verts)
        op, _, _ = _ptr(offsets)
        fp, _, _ = _ptr(root_first)
        nc, nv = ctypes.c_int64(), ctypes.c_int64()
        size = (lambda a: int(a.numel() if _is_torch(a) else np.asarray(a).size))
        st = lib().cc_enumerate_by_roots(self.h, vp, size(verts), op, max(size(offsets) - 1, 0),
                                         fp, size(root_first), ctypes.byref(nc), ctypes.byref(nv))
        if st == CC_ERR_INTERNAL:
            _check(st, "cc_enumerate_by_roots", self._info_fn)
        if st != CC_OK:
            err = CCError(st, "cc_enumerate_by_roots")
            err.required = (nc.value, nv.value)
            raise err
        return nc.value, nv.value

    def pages_by_roots(self, max_verts: int, max_cycles: int | None = None, device="cuda",
                       one_run: bool | None = None):
        """Yield (root_lo, root_hi, verts, offsets): the whole output in pages
        of consecutive root ranges, each holding at most max_verts vertex ids
        (and max_cycles cycles), offsets from 0 in each page.

        When the output fits device memory twice over (or one_run=True), one
        run enumerates everything grouped by root (cc_enumerate_by_roots) and
        the pages are copied out of it: ranges chosen greedily from the
        roots' exact sizes.  Otherwise (or one_run=False) each page is a run
        of its own over its roots (cc_enumerate_roots), the ranges starting
        from an even split sized by the whole histogram and halved when
        their cycles do not fit; no page reruns the whole graph.  With device
        output every page is written into the same two buffers of the page
        limits (the arrays yielded are views of them, valid until the next
        page; in the one-run form the ids are a view of the grouped output);
        with host output each page gets arrays of its exact size.
        Raises ValueError if the cycles of a single root do not fit."""
        total = self.root_total()
        if total == 0:
            return
        want = self._sizes()
        nv_all = int((want * np.arange(want.size)).sum())
        nc_all = int(want.sum())
        cyc_cap = max_cycles if max_cycles is not None else max_verts // 3
        if one_run is None:
            need = 2 * (4 * nv_all + 8 * (nc_all + 1)) + 16 * nc_all + 8 * (total + 1)
            if self.output_device:
                import torch
                free, _ = torch.cuda.mem_get_info()
            else:
                free = 0  # host output keeps the whole output in host memory: per-range runs
            one_run = need + (256 << 20) <= free
        if one_run:
            yield from self._pages_one_run(total, nc_all, nv_all, max_verts, cyc_cap, device)
            return
        yield from self._pages_by_range_runs(total, nv_all, max_verts, cyc_cap, device)

    def _pages_one_run(self, total, nc_all, nv_all, max_verts, cyc_cap, device):
        if self.output_device:
            import torch
            gv = torch.empty(max(nv_all, 1), dtype=torch.int32, device=device)
            go = torch.empty(nc_all + 1, dtype=torch.int64, device=device)
            gf = torch.empty(total + 1, dtype=torch.int64, device=device)
        else:
            gv = np.empty(max(nv_all, 1), np.int32)
            go = np.empty(nc_all + 1, np.int64)
            gf = np.empty(total + 1, np.int64)
        self.enumerate_by_roots_into(gv, go, gf)
        if self.output_device:
            both = torch.cat((gf, go[gf])).cpu().numpy()  # one copy back
            first, vpos = both[:total + 1], both[total + 1:]
            offs = torch.empty(cyc_cap + 1, dtype=torch.int64, device=device)
        else:
            first = gf
            vpos = go[gf]
        lo = 0
        while lo < total:
            # the longest range from lo that fits the page limits
            hi_v = int(np.searchsorted(vpos, vpos[lo] + max_verts, side="right")) - 1
            hi_c = int(np.searchsorted(first, first[lo] + cyc_cap, side="right")) - 1
            hi = min(hi_v, hi_c, total)
            if hi <= lo:
                c0, c1 = int(first[lo]), int(first[lo + 1])
                raise ValueError(f"the {c1 - c0} cycles of root {lo} need "
                                 f"{int(vpos[lo + 1] - vpos[lo])} vertex ids, more than "
                                 f"max_verts={max_verts}")
            c0, c1 = int(first[lo]), int(first[hi])
            v0, v1 = int(vpos[lo]), int(vpos[hi])
            if self.output_device:
                # the page's ids in place; its offsets from 0 in the page buffer
                torch.sub(go[c0:c1 + 1], v0, out=offs[:c1 - c0 + 1])
                yield lo, hi, gv[v0:v1], offs[:c1 - c0 + 1]
            else:
                yield lo, hi, gv[v0:v1].copy(), go[c0:c1 + 1] - v0
            lo = hi

    def _pages_by_range_runs(self, total, nv_all, max_verts, cyc_cap, device):
        parts = max(1, -(-nv_all // max(max_verts, 1)))
        bounds = [total * i // parts for i in range(parts + 1)]
        todo = [(bounds[i], bounds[i + 1]) for i in range(parts) if bounds[i] < bounds[i + 1]]
        if self.output_device:
            import torch
            verts = torch.empty(max(max_verts, 1), dtype=torch.int32, device=device)
            offs = torch.empty(cyc_cap + 1, dtype=torch.int64, device=device)
        while todo:
            lo, hi = todo.pop(0)
            if not self.output_device:
                # host buffers: the library sizes the range by a counting run
                h = self.histogram_roots(lo, hi)
                nc, nv = int(h.sum()), int((h * np.arange(h.size)).sum())
                fits = nv <= max_verts and nc <= cyc_cap
                if fits:
                    verts = np.empty(max(nv, 1), np.int32)
                    offs = np.empty(nc + 1, np.int64)
                    self.enumerate_roots_into(lo, hi, verts, offs)
            else:
                try:
                    nc, nv = self.enumerate_roots_into(lo, hi, verts, offs)
                    fits = True
                except CCError as e:
                    if e.status != CC_ERR_BUFFER_TOO_SMALL:
                        raise
                    nc, nv = e.required
                    fits = False
            if not fits:
                if hi - lo == 1:
                    raise ValueError(f"the {nc} cycles of root {lo} need {nv} vertex ids, "
                                     f"more than max_verts={max_verts}")
                mid = (lo + hi) // 2
                todo[:0] = [(lo, mid), (mid, hi)]
                continue
            yield lo, hi, verts[:nv], offs[:nc + 1]

    def labels(self) -> np.ndarray:
        lab = np.zeros(max(self.n, 1), np.int32)
        _check(lib().cc_labels(self.h, ctypes.c_void_p(lab.ctypes.data)), "cc_labels")
        return lab[:self.n]

    def frontier(self) -> np.ndarray:
        f = np.zeros(self.n + 1, np.int64)
        _check(lib().cc_frontier(self.h, ctypes.c_void_p(f.ctypes.data), f.size), "cc_frontier")
        return f

    def level_times(self) -> np.ndarray:
        """Per-level device ms of the last call made with profile=True."""
        a = np.zeros(self.n + 1, np.float64)
        _check(lib().cc_level_times(self.h, ctypes.c_void_p(a.ctypes.data), a.size), "cc_level_times")
        return a

    def last_run(self) -> dict:
        info = RunInfo()
        _check(lib().cc_last_run(self.h, ctypes.byref(info)), "cc_last_run")
        return info.as_dict()


def _as_i32(x):
    if x is None:
        return None
    if _is_torch(x):
        import torch
        if x.dtype != torch.int32:
            x = x.to(torch.int32)
        return x if x.is_contiguous() else x.contiguous()
    a = np.asarray(x)
    if a.size == 0:
        a = np.zeros(1, np.int32)
    return np.ascontiguousarray(a, dtype=np.int32)


def prepare(g, **kw) -> Graph:
    """cc_prepare on a graphgen.CSR-like object (n, row_ptr, col_idx)."""
    return Graph(g.n, g.row_ptr, g.col_idx, **kw)


class Batch:
    """Many graphs packed as one CSR (cc_prepare_batch)."""

    def __init__(self, graph_vtx_off, row_ptr, col_idx, stream=None, budget_bytes: int = 0,
                 dfs_waves_per_cu: int = 0, dfs_donate_min: int = 0, dfs_claim: int = 0,
                 profile: bool = False, sizes=None):
        L = lib()
        off, off_dev, k0 = _ptr(_as_i32(graph_vtx_off))
        rp, rp_dev, k1 = _ptr(_as_i32(row_ptr))
        ci, ci_dev, k2 = _ptr(_as_i32(col_idx))
        if not (off_dev == rp_dev == ci_dev):
            raise ValueError("batch arrays must all be host or all be device")
        self.n_graphs = int((graph_vtx_off.numel() if _is_torch(graph_vtx_off)
                             else np.asarray(graph_vtx_off).size) - 1)
        if sizes is None:  # graph sizes on the host (pass them to skip a device read)
            sizes = np.diff(np.asarray(graph_vtx_off.cpu() if _is_torch(graph_vtx_off)
                                       else graph_vtx_off, dtype=np.int64))
        self.sizes = np.asarray(sizes, dtype=np.int64)
        self.n_vertices = int(self.sizes.sum())
        self.max_n = int(self.sizes.max()) if self.sizes.size else 0
        flags = CC_INPUT_DEVICE if off_dev else 0
        if profile:
            flags |= CC_PROFILE
        self.opt = Options(_stream_handle(stream), int(budget_bytes), flags, 0,
                           int(dfs_waves_per_cu), 0, int(dfs_donate_min), int(dfs_claim))
        h = ctypes.c_void_p()
        st = L.cc_prepare_batch(self.n_graphs, off, rp, ci, ctypes.byref(self.opt), ctypes.byref(h))
        _check(st, "cc_prepare_batch")
        self.h = h

    def release(self):
        if getattr(self, "h", None):
            lib().cc_release_batch(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.release()

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass

    def histograms(self, per_graph_launch: bool = False) -> np.ndarray:
        """[n_graphs, max_n + 1] int64: row g is graph g's histogram (zero past
        the graph's own n + 1 entries)."""
        stride = self.max_n + 1
        out = np.zeros((self.n_graphs, stride), np.int64)
        off = np.arange(self.n_graphs, dtype=np.int64) * stride
        self.histograms_into(out.reshape(-1), off, per_graph_launch)
        return out

    def histograms_into(self, hists: np.ndarray, hist_off: np.ndarray,
                        per_graph_launch: bool = False) -> None:
        """cc_histogram_batch: graph g's histogram (n_g + 1 entries) into
        hists[hist_off[g]:]; `hists` is a host int64 array covering every
        range, `hist_off` int64 offsets."""
        hists = np.asarray(hists)
        if hists.dtype != np.int64 or not hists.flags.c_contiguous:
            raise ValueError("hists must be a contiguous int64 array")
        off = np.ascontiguousarray(hist_off, dtype=np.int64)
        if off.size != self.n_graphs:
            raise ValueError("hist_off needs one offset per graph")
        if off.size and (off.min() < 0 or (off + self.sizes + 1).max() > hists.size):
            raise ValueError("a graph's histogram range falls outside hists")
        hp = ctypes.c_void_p(hists.ctypes.data)
        op = ctypes.c_void_p(off.ctypes.data)
        if per_graph_launch:
            st = lib().cc_histogram_batch_mode(self.h, hp, op, CC_BATCH_PER_GRAPH)
        else:
            st = lib().cc_histogram_batch(self.h, hp, op)
        _check(st, "cc_histogram_batch", lambda p: lib().cc_batch_last_run(self.h, p))

    def labels(self) -> np.ndarray:
        lab = np.zeros(max(self.n_vertices, 1), np.int32)
        _check(lib().cc_batch_labels(self.h, ctypes.c_void_p(lab.ctypes.data)), "cc_batch_labels")
        return lab[:self.n_vertices]

    def last_run(self) -> dict:
        info = RunInfo()
        _check(lib().cc_batch_last_run(self.h, ctypes.byref(info)), "cc_batch_last_run")
        return info.as_dict()


def prepare_batch(batch, **kw) -> Batch:
    """cc_prepare_batch on a graphgen.Batch-like object."""
    return Batch(batch.graph_vtx_off, batch.row_ptr, batch.col_idx, **kw)


class Server:
    """Request loop over many independent graphs (cc_server_*).  submit()
    copies the graph and returns a request id at once; result() waits for
    that request and returns (histogram, latency_ms, status)."""

    def __init__(self, slots: int = 0, max_batch_graphs: int = 0, slot_root_slots: int = 0,
                 slot_work_bytes: int = 0, dfs_waves_per_cu: int = 0):
        L = lib()
        self.opt = ServerOptions(int(slots), int(max_batch_graphs), int(slot_root_slots),
                                 int(slot_work_bytes), int(dfs_waves_per_cu), 0)
        h = ctypes.c_void_p()
        _check(L.cc_server_create(ctypes.byref(self.opt), ctypes.byref(h)), "cc_server_create")
        self.h = h
        self._n = {}

    def submit(self, n, row_ptr, col_idx) -> int:
        rp = np.ascontiguousarray(np.asarray(row_ptr), dtype=np.int32)
        ci = np.ascontiguousarray(np.asarray(col_idx), dtype=np.int32)
        if ci.size == 0:
            ci = np.zeros(1, np.int32)
        rid = ctypes.c_int64()
        _check(lib().cc_server_submit(self.h, int(n), ctypes.c_void_p(rp.ctypes.data),
                                      ctypes.c_void_p(ci.ctypes.data), ctypes.byref(rid)),
               "cc_server_submit")
        self._n[rid.value] = int(n)
        return rid.value

    def submit_graph(self, g) -> int:
        return self.submit(g.n, g.row_ptr, g.col_idx)

    def result(self, request_id: int, timeout_s: float = 60.0):
        """(hist int64[n+1], latency_ms, status).  Raises CCError(CC_ERR_NOT_READY)
        on timeout; `status` is the request's own (0, or e.g. CC_ERR_NOT_SIMPLE)."""
        n = self._n[request_id]
        hist = np.zeros(n + 1, np.int64)
        lat = ctypes.c_double()
        rst = ctypes.c_int()
        _check(lib().cc_server_result(self.h, int(request_id), float(timeout_s),
                                      ctypes.c_void_p(hist.ctypes.data), n + 1,
                                      ctypes.byref(lat), ctypes.byref(rst)), "cc_server_result")
        del self._n[request_id]
        return hist, lat.value, rst.value

    def stats(self) -> dict:
        a = np.zeros(5, np.int64)
        _check(lib().cc_server_stats(self.h, ctypes.c_void_p(a.ctypes.data), 5), "cc_server_stats")
        return {"completed": int(a[0]), "batches": int(a[1]), "pending": int(a[2]),
                "rejected": int(a[3]), "max_batch": int(a[4])}

    def close(self):
        if getattr(self, "h", None):
            lib().cc_server_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
