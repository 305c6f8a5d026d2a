"""Host-only build of the graph-build and serving-allocator code under
AddressSanitizer and UndefinedBehaviorSanitizer (no GPU): problem images,
union plans and workspace layouts of random problems are checked for their
invariants, and the serving arena's range allocator against a byte-map model,
including the admission order (image placed while the batch workspace is
held, the grown workspace placed afterwards).  tests/native/host_check.cc
holds the checks; the kernel launchers are stubs that abort if reached.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def test_graph_build_and_arena_allocator_under_sanitizers(tmp_path):
    cxx = shutil.which("g++")
    if cxx is None or not os.path.exists(os.path.join(ROCM, "include", "hip", "hip_runtime.h")):
        pytest.skip("g++ or the HIP headers are missing")
    exe = str(tmp_path / "host_check")
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]
    cmd = [cxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer"] + san + [
        "-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(ROCM, "include"),
        "-I" + os.path.join(ROOT, "include"),
        "-I" + os.path.join(ROOT, "paper_2509_26581_amd", "csrc"),
        os.path.join(ROOT, "tests", "native", "host_check.cc"),
        "-L" + os.path.join(ROCM, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(ROCM, "lib"),
        "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, timeout=600)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    res = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "host checks passed" in res.stdout
