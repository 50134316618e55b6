"""Host code under sanitizers, on the CPU (no GPU): the library's host-side
table construction and C-ABI argument handling (plan.cpp, capi.cpp,
ckks.cpp, timing.cpp) under AddressSanitizer + UndefinedBehaviorSanitizer
(LeakSanitizer at exit), a workspace audit of every CKKS operation
(exactly sized buffers, kernel stand-ins that touch the ends of every range
a launch uses), the request dispatcher's threads, queues, batching
and event reference counts (server.cpp) under ThreadSanitizer with
stand-in key switching, and the C oracle under ASan + UBSan.  The host
sources are compiled against a stand-in HIP runtime (tests/sanitize/fakehip:
host memory, synchronous kernels) with the kernel launchers stubbed
(tests/sanitize/kernel_stubs.cpp)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_2212_14191_amd", "csrc")
CXX = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-I" + os.path.join(SAN, "fakehip"),
       "-I" + os.path.join(ROOT, "include")]

pytestmark = pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None,
                                reason="needs gcc / g++")


def build_and_run(cmd, exe, env_extra=None):
    r = subprocess.run(cmd + ["-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, **(env_extra or {}))
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-6000:]
    assert "Sanitizer" not in out and "runtime error" not in out, out[-6000:]
    return r.stdout


def test_host_tables_under_asan_ubsan(tmp_path):
    srcs = [os.path.join(CSRC, f) for f in ("plan.cpp", "capi.cpp", "ckks.cpp", "timing.cpp")]
    srcs += [os.path.join(SAN, "kernel_stubs.cpp"), os.path.join(SAN, "tables_driver.cpp")]
    out = build_and_run(CXX + ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-x", "c++"]
                        + srcs + ["-lpthread"], str(tmp_path / "tables"),
                        {"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0"})
    assert "0 failures" in out


def test_workspace_audit_under_asan(tmp_path):
    """Every CKKS operation with buffers of exactly the size the C ABI asks
    for, the kernel stand-ins touching the ends of every range the real
    launches use: an undersized workspace region is a sanitizer report."""
    srcs = [os.path.join(CSRC, f) for f in ("plan.cpp", "capi.cpp", "ckks.cpp", "timing.cpp")]
    srcs += [os.path.join(SAN, "kernel_stubs.cpp"), os.path.join(SAN, "ws_audit_driver.cpp")]
    out = build_and_run(CXX + ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-x", "c++"]
                        + srcs + ["-lpthread"], str(tmp_path / "audit"),
                        {"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0"})
    assert " 0 failures" in out


def test_dispatcher_under_tsan(tmp_path):
    srcs = [os.path.join(CSRC, f) for f in ("server.cpp", "capi.cpp", "plan.cpp", "timing.cpp")]
    srcs += [os.path.join(SAN, f) for f in ("kernel_stubs.cpp", "fake_keyswitch.cpp", "server_driver.cpp")]
    out = build_and_run(CXX + ["-fsanitize=thread", "-x", "c++"] + srcs + ["-lpthread"], str(tmp_path / "server"),
                        {"TSAN_OPTIONS": "halt_on_error=1"})
    assert "0 wrong" in out


def test_oracle_under_asan_ubsan(tmp_path):
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-fopenmp", os.path.join(ROOT, "oracle", "oracle.c"),
           os.path.join(SAN, "oracle_driver.c")]
    out = build_and_run(cmd, str(tmp_path / "oracle"))
    assert "0 failures" in out
