"""The library's host code (argument validation, workspace layout and error
returns of the C ABI in include/ep_tv.h and include/ep_tv_net.h) under
AddressSanitizer, on the CPU: api.cpp, net.hip and noalloc.hip are compiled with
the sanitizer on their host side only (device code is unchanged), linked with
the library's other objects and the driver tests/asan_abi_driver.cpp, whose
calls all return before any device call.  The test fails on any sanitizer
report (out-of-bounds access, use after free, leak) or failed expectation."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
from paper_2110_01585_amd import build as B  # noqa: E402

INSTRUMENTED = ("api.cpp", "net.hip", "noalloc.hip")
ASAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
        "-fno-omit-frame-pointer", "-g"]


def _hipcc():
    try:
        return B._hipcc()
    except RuntimeError:
        pytest.skip("hipcc not available")


def test_abi_host_code_under_asan(tmp_path):
    hipcc = _hipcc()
    srcs = B.sources()
    # the other objects as the library is built (compiled here if missing)
    plain = [s for s in srcs if os.path.basename(s) not in INSTRUMENTED]
    objs = []
    for s in plain:
        o = os.path.join(B.BUILD, os.path.basename(s) + ".o")
        if not os.path.exists(o) or os.path.getmtime(o) < os.path.getmtime(s):
            os.makedirs(B.BUILD, exist_ok=True)
            o = B._compile(s)
        objs.append(o)
    for name in INSTRUMENTED:
        src = os.path.join(B.CSRC, name)
        o = str(tmp_path / (name + ".asan.o"))
        r = subprocess.run([hipcc, "-c", src, "-o", o, f"-I{B.INCLUDE}"] + B.COMMON + ASAN,
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        objs.append(o)
    exe = str(tmp_path / "asan_abi")
    drv = os.path.join(ROOT, "tests", "asan_abi_driver.cpp")
    drv_o = str(tmp_path / "asan_abi_driver.o")
    r = subprocess.run([hipcc, "-c", drv, "-o", drv_o, f"-I{B.INCLUDE}", "-O1"] + B.COMMON + ASAN,
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    r = subprocess.run([hipcc, "-o", exe, drv_o] + objs + [f"--offload-arch={B.ARCH}"] + ASAN,
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    print(r.stdout[-2000:])
    assert "ERROR: AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    assert "ERROR: LeakSanitizer" not in r.stderr, r.stderr[-4000:]
    assert "runtime error" not in r.stderr, r.stderr[-4000:]
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-2000:])
    assert r.stdout.strip().splitlines()[-1].startswith("ok:")
