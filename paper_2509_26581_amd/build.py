"""Build the gfx950 solver library (libgba.so) in-tree with hipcc.

Usage: python -m paper_2509_26581_amd.build   (or build() from Python).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = ["gba_kernels.hip", "gba_host.hip", "gba_api.hip", "gba_serve.hip", "gba_vi.hip"]
LIB = os.path.join(HERE, "libgba.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(HERE, "csrc")]


def build(verbose=False, lib=LIB, defines=()):
    out_dir = os.path.join(ROOT, "_build", os.path.basename(lib).replace(".so", ""))
    os.makedirs(out_dir, exist_ok=True)
    objs = []
    for src in SRC:
        obj = os.path.join(out_dir, src.replace(".hip", ".o"))
        cmd = [HIPCC] + FLAGS + ["-D" + d for d in defines] + [
            "-c", os.path.join(HERE, "csrc", src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = lib + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
