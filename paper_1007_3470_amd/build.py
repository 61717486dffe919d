"""Build the gfx950 shared library libhfgpe.so in-tree with hipcc."""
from __future__ import annotations

import concurrent.futures
import glob
import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "libhfgpe.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compile every .hip source (in parallel, one object each) and link
    libhfgpe.so (always rebuilds)."""
    srcs = sources()
    objdir = tempfile.mkdtemp(prefix="hfgpe_build_")
    try:
        objs = [os.path.join(objdir, os.path.basename(s)[:-4] + ".o") for s in srcs]
        cmds = [[HIPCC] + FLAGS + ["-I", INCLUDE, "-I", CSRC, "-c", "-o", o, s] for s, o in zip(srcs, objs)]
        if verbose:
            for c in cmds:
                print(" ".join(c), flush=True)
        n = jobs or min(len(cmds), os.cpu_count() or 1, 8)
        with concurrent.futures.ThreadPoolExecutor(max_workers=n) as ex:
            for f in [ex.submit(subprocess.check_call, c) for c in cmds]:
                f.result()
        tmp = LIB + ".tmp%d" % os.getpid()
        link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
        if verbose:
            print(" ".join(link), flush=True)
        subprocess.check_call(link)
        os.replace(tmp, LIB)
    finally:
        shutil.rmtree(objdir, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
