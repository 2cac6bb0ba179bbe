"""Build libdash.so (the C-ABI library) for gfx950 with hipcc, in-tree.

Each source is compiled to an object of its own, in parallel, and the
objects are linked into the shared library."""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdash.so")
SOURCES = [os.path.join(CSRC, f) for f in
           ("dash_host.cpp", "dash_server.cpp", "dash_kernels.hip", "dash_split.hip", "dash_init.hip",
            "dash_anomaly.hip", "dash_noalloc.hip")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 instructions anywhere in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
    "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    return r, cmd


def build(verbose: bool = False) -> str:
    """Compile every source (always) and link libdash.so."""
    with tempfile.TemporaryDirectory(prefix="dash_build_") as tmpd:
        objs = [os.path.join(tmpd, os.path.basename(src) + ".o") for src in SOURCES]
        cmds = [[HIPCC, *FLAGS, "-c", src, "-o", obj] for src, obj in zip(SOURCES, objs)]
        with ThreadPoolExecutor(max_workers=len(cmds)) as ex:
            results = list(ex.map(lambda c: _run(c, verbose), cmds))
        failed = False
        for r, cmd in results:
            msg = r.stdout + r.stderr
            msg = "\n".join(l for l in msg.splitlines() if "packed-fp32-ops" not in l)
            if r.returncode != 0:
                failed = True
                sys.stderr.write(msg + "\n")
            elif verbose and msg.strip():
                sys.stderr.write(msg + "\n")
        if failed:
            raise RuntimeError("hipcc failed building libdash.so")
        tmp = LIB + ".tmp"
        r, _ = _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs], verbose)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError("linking libdash.so failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
