"""Host-side checks of the C ABI: the library loads, exports every entry
point include/cc.h declares, lays out its structs as the header does, and
rejects bad arguments before touching a device.  No GPU needed."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cc.h")


@pytest.fixture(scope="module")
def L():
    from paper_1410_4876_amd import cc
    if not os.path.exists(cc.LIB_PATH):
        from paper_1410_4876_amd import build
        build.build()
    return cc.lib()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cc_[a-z_]+)\s*\(", text)))


def test_header_declares_the_core_calls():
    names = declared_functions()
    for must in ["cc_prepare", "cc_count", "cc_histogram", "cc_enumerate", "cc_release",
                 "cc_status_string"]:
        assert must in names


def test_every_declared_symbol_is_exported(L):
    out = subprocess.check_output(["nm", "-D", "--defined-only",
                                   os.path.join(ROOT, "paper_1410_4876_amd", "libcc.so")]).decode()
    exported = set(re.findall(r" T (cc_\w+)", out))
    missing = [f for f in declared_functions() if f not in exported]
    assert not missing, missing


def test_status_strings_and_version(L):
    from paper_1410_4876_amd import cc
    assert L.cc_abi_version() == 2
    for code in range(-9, 1):
        assert cc.status_string(code) and cc.status_string(code) != "unknown status"
    assert cc.status_string(-99) == "unknown status"


def test_struct_layout_matches_header(tmp_path):
    from paper_1410_4876_amd import cc
    src = tmp_path / "layout.c"
    src.write_text('#include <stddef.h>\n#include <stdio.h>\n#include "cc.h"\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(cc_options),'
                   ' offsetof(cc_options, frontier_budget_bytes), offsetof(cc_options, flags),'
                   ' offsetof(cc_options, bfs_blocks), sizeof(cc_run_info),'
                   ' offsetof(cc_run_info, switch_level), offsetof(cc_run_info, gpu_ms),'
                   ' offsetof(cc_run_info, head_steps), offsetof(cc_run_info, head_bytes));return 0;}\n')
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = list(map(int, subprocess.check_output([str(exe)]).split()))
    want = [ctypes.sizeof(cc.Options), cc.Options.frontier_budget_bytes.offset,
            cc.Options.flags.offset, cc.Options.bfs_blocks.offset, ctypes.sizeof(cc.RunInfo),
            cc.RunInfo.switch_level.offset, cc.RunInfo.gpu_ms.offset,
            cc.RunInfo.head_steps.offset, cc.RunInfo.head_bytes.offset]
    assert got == want


def test_argument_errors_before_any_device_call(L):
    from paper_1410_4876_amd import cc
    h = ctypes.c_void_p()
    rp = (ctypes.c_int32 * 3)(0, 1, 2)
    ci = (ctypes.c_int32 * 2)(1, 0)
    assert L.cc_prepare(-1, rp, ci, None, ctypes.byref(h)) == cc.CC_ERR_INVALID_ARG
    assert L.cc_prepare(1025, rp, ci, None, ctypes.byref(h)) == cc.CC_ERR_TOO_LARGE
    assert L.cc_prepare(2, rp, ci, None, None) == cc.CC_ERR_INVALID_ARG
    assert L.cc_prepare(2, None, ci, None, ctypes.byref(h)) == cc.CC_ERR_INVALID_ARG
    bad = cc.Options(None, 0, 1 << 7, 0, 0, 0, 0, 0)
    assert L.cc_prepare(2, rp, ci, ctypes.byref(bad), ctypes.byref(h)) == cc.CC_ERR_INVALID_ARG
    neg = cc.Options(None, -5, 0, 0, 0, 0, 0, 0)
    assert L.cc_prepare(2, rp, ci, ctypes.byref(neg), ctypes.byref(h)) == cc.CC_ERR_INVALID_ARG
    neg_claim = cc.Options(None, 0, 0, 0, 0, 0, 0, -64)
    assert L.cc_prepare(2, rp, ci, ctypes.byref(neg_claim), ctypes.byref(h)) == cc.CC_ERR_INVALID_ARG
    forced = cc.Options(None, 0, cc.CC_FORCE_DFS, 2, 0, 0, 0, 0)
    assert L.cc_prepare(2, rp, ci, ctypes.byref(forced), ctypes.byref(h)) == cc.CC_ERR_INVALID_ARG
    # host CSR whose header cannot describe a simple graph
    rp_bad = (ctypes.c_int32 * 3)(1, 1, 2)
    assert L.cc_prepare(2, rp_bad, ci, None, ctypes.byref(h)) == cc.CC_ERR_NOT_SIMPLE
    rp_big = (ctypes.c_int32 * 3)(0, 2, 5)
    assert L.cc_prepare(2, rp_big, ci, None, ctypes.byref(h)) == cc.CC_ERR_NOT_SIMPLE
    assert not h.value
    # calls on a null handle
    total = ctypes.c_int64()
    assert L.cc_count(None, ctypes.byref(total)) == cc.CC_ERR_INVALID_ARG
    nc, nv = ctypes.c_int64(), ctypes.c_int64()
    offs = (ctypes.c_int64 * 2)()
    assert L.cc_enumerate_lengths(None, 3, 5, None, 0, offs, 1, ctypes.byref(nc),
                                  ctypes.byref(nv)) == cc.CC_ERR_INVALID_ARG
    first = (ctypes.c_int64 * 2)()
    assert L.cc_enumerate_by_roots(None, None, 0, offs, 1, first, 2, ctypes.byref(nc),
                                   ctypes.byref(nv)) == cc.CC_ERR_INVALID_ARG
    L.cc_release(None)
    # batch calls on a null handle
    hists = (ctypes.c_int64 * 4)()
    hoff = (ctypes.c_int64 * 1)(0)
    assert L.cc_histogram_batch(None, hists, hoff) == cc.CC_ERR_INVALID_ARG
    assert L.cc_histogram_batch_mode(None, hists, hoff, 0) == cc.CC_ERR_INVALID_ARG


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_1410_4876_amd import cc
    monkeypatch.setattr(cc, "_lib", None)
    monkeypatch.setattr(cc, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        cc.lib()
