"""The serving admission policy on the CPU: a C++ check program built with
g++ against the policy header (no HIP), plus host-side argument checks of
the server entry points that fail before any device is touched."""
import ctypes
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_admission_policy(tmp_path):
    exe = tmp_path / "serve_policy_check"
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-Wall", "-Werror",
                           "-I", os.path.join(ROOT, "paper_1410_4876_amd", "csrc"),
                           os.path.join(ROOT, "tests", "native", "serve_policy_check.cpp"),
                           "-o", str(exe)])
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout + out.stderr


@pytest.fixture(scope="module")
def L():
    from paper_1410_4876_amd import cc
    if not os.path.exists(cc.LIB_PATH):
        from paper_1410_4876_amd import build
        build.build()
    return cc.lib()


def test_server_argument_errors(L):
    from paper_1410_4876_amd import cc
    assert L.cc_server_create(None, None) == cc.CC_ERR_INVALID_ARG
    h = ctypes.c_void_p()
    bad = cc.ServerOptions(-1, 0, 0, 0, 0, 0)
    assert L.cc_server_create(ctypes.byref(bad), ctypes.byref(h)) == cc.CC_ERR_INVALID_ARG
    assert not h.value
    rid = ctypes.c_int64()
    assert L.cc_server_submit(None, 3, None, None, ctypes.byref(rid)) == cc.CC_ERR_INVALID_ARG
    hist = (ctypes.c_int64 * 4)()
    assert L.cc_server_result(None, 1, 0.0, hist, 4, None, None) == cc.CC_ERR_INVALID_ARG
    assert L.cc_server_stats(None, hist, 4) == cc.CC_ERR_INVALID_ARG
    L.cc_server_destroy(None)
    assert cc.status_string(cc.CC_ERR_NOT_READY) == "request not finished yet"
