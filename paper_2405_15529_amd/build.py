"""Build the gfx950 shared library ``libpylom.so`` in-tree with hipcc.

Each source is compiled to an object in parallel (every kernel is launched
from the file that defines it, so no relocatable device code is needed),
then the objects are linked into the shared library.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libpylom.so")
SOURCES = ["abi.hip", "tsqr.hip", "svd.hip", "misc.hip", "refine.hip", "spod.hip", "ctsqr.hip",
           "blocked.hip", "dmd.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed-FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed: {' '.join(cmd[-3:])}")


def _stale(obj: str, src: str, headers) -> bool:
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(f) > t for f in [src, *headers])


def build(verbose: bool = False, jobs: int | None = None, incremental: bool = False) -> str:
    """Compile every source (or, with incremental, only those whose object is
    older than the source or a header) and link libpylom.so."""
    os.makedirs(OBJ, exist_ok=True)
    inc_dir = os.path.join(HERE, "..", "include")
    inc = ["-I", inc_dir]
    headers = [os.path.join(CSRC, h) for h in os.listdir(CSRC) if h.endswith(".hpp")]
    headers += [os.path.join(inc_dir, h) for h in os.listdir(inc_dir) if h.endswith(".h")]
    objs = []
    cmds = []
    for s in SOURCES:
        o = os.path.join(OBJ, s.replace(".hip", ".o"))
        src = os.path.join(CSRC, s)
        objs.append(o)
        if incremental and not _stale(o, src, headers):
            continue
        cmds.append([HIPCC, *FLAGS, *inc, "-c", "-o", o, src])
    jobs = jobs or max(1, min(len(cmds), 8, os.cpu_count() or 1))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        for f in [ex.submit(_run, c, verbose) for c in cmds]:
            f.result()
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, incremental="--incremental" in sys.argv))
