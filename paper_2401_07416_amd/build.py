"""Build libtdse.so in-tree with hipcc for gfx950.

The half-step kernel instances are split over several translation units
(one per precision and vector width) that compile in parallel, then link
with the runtime into one shared library."""
from __future__ import annotations

import glob
import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libtdse.so")
OBJ = os.path.join(HERE, "_build")
ARCH = os.environ.get("TDSE_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # no packed FP32 instructions: the compiler may not form them
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # every multiply and add rounded on its own, as written: the one-pass and
    # two-pass kernels then give the same bits, and FP64 follows the
    # oracle's rounding sequence
    "-ffp-contract=off",
    "-Wno-unused-command-line-argument",
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def build(verbose: bool = False, extra=(), jobs: int = 8) -> str:
    os.makedirs(OBJ, exist_ok=True)
    t0 = time.time()
    procs = []
    objs = []
    for src in sources():
        obj = os.path.join(OBJ, os.path.basename(src)[:-4] + ".o")
        objs.append(obj)
        cmd = ["hipcc", *FLAGS, *extra, "-c", src, "-o", obj]
        while len([p for p in procs if p[0].poll() is None]) >= jobs:
            time.sleep(0.2)
        procs.append((subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                                       text=True), src))
    failed = False
    for p, src in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            failed = True
            sys.stderr.write(f"--- {src}\n{out}\n")
    if failed:
        raise RuntimeError("hipcc failed building libtdse.so")
    tmp = OUT + ".tmp"
    subprocess.check_call(["hipcc", "-shared", f"--offload-arch={ARCH}", *objs, "-o", tmp])
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT} in {time.time() - t0:.1f}s")
    return OUT


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
