"""Builds libladlasso.so (HIP, gfx950) in-tree with hipcc."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libladlasso.so")

SOURCES = ["ladl_solve_wave.hip", "ladl_solve_tile.hip", "ladl_solve_plain.hip", "ladl_cv.hip", "ladl_brute.hip", "ladl_noalloc.hip",
           "ladl_api.cpp"]

FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
    # no packed fp32 instructions in device code (the host pass warns that
    # it does not know the feature)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def build(verbose: bool = False, extra=(), out: str = LIB) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    bdir = os.path.join(CSRC, "_build")
    os.makedirs(bdir, exist_ok=True)
    objs = [os.path.join(bdir, src + ".o") for src in SOURCES]
    cmds = [[hipcc, *FLAGS, *extra, "-x", "hip", "-c", os.path.join(CSRC, src), "-I", os.path.join(ROOT, "include"),
             "-I", CSRC, "-o", obj] for src, obj in zip(SOURCES, objs)]
    for cmd in cmds:
        if verbose:
            print(" ".join(cmd), flush=True)
    # the translation units compile side by side (the wavefront kernel's
    # variants dominate the build time)
    jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", "0")) or (os.cpu_count() or 1)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        codes = list(ex.map(subprocess.call, cmds))
    for cmd, rc in zip(cmds, codes):
        if rc != 0:
            raise subprocess.CalledProcessError(rc, cmd)
    tmp = out + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-fPIC", "-shared", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
