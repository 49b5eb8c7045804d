"""The host layout builder (csrc/layout.cpp) under AddressSanitizer and
UndefinedBehaviorSanitizer: tests/sanitize/layout_check.cpp, built with g++
(host code only, no GPU), builds the pull layout with and without delay
phases, its 4-byte compact records, the lane-only layout and its lane
records, the slice partitions and the push layout of empty nets, nets with
duplicates, self-loops and signed-zero weights, hub nets whose posts
overflow the lane-owned rows, delays up to 64 and 2^20 neurons, and checks
the invariants the kernels rely on (every record field decoded back)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_layout_builder_under_sanitizers(tmp_path):
    exe = tmp_path / "layout_check"
    # the sanitizer runtimes are linked statically, so they need not come first
    # among the process's shared libraries
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-static-libasan", "-static-libubsan", "-D__HIP_PLATFORM_AMD__",
           "-I/opt/rocm/include",
           os.path.join(HERE, "sanitize", "layout_check.cpp"),
           os.path.join(ROOT, "paper_2305_02510_amd", "csrc", "layout.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert res.returncode == 0, res.stdout[-2000:] + res.stderr[-4000:]
    assert res.stdout.startswith("ok "), res.stdout
