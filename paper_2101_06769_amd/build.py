"""Build libmplb.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2101_06769_amd.build
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmplb.so")
SOURCES = ["k_step.hip", "k_nphi.hip", "k_host.hip", "k_batch.hip", "api.cpp"]

# hipcc flags: gfx950 only, C++20, no packed-FP32 instructions, and
# multiply-add fusion only within one source expression (-ffp-contract=on):
# the backend would otherwise fuse across statements wherever they share a
# basic block, so kernels that differ only in control flow (per-lane and
# row-form addressing, solo and batched launches) would round differently.
HIPCC_FLAGS = ["--offload-arch=gfx950", "-std=c++20", "-O3", "-fPIC", "-shared",
               "-ffp-contract=on",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-Wall", "-Wno-unused-command-line-argument"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(args, target, verbose):
    tmp = target + ".tmp%d" % os.getpid()
    cmd = [hipcc()] + args + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    os.replace(tmp, target)


def build(verbose: bool = False) -> str:
    """Compile every source to an object in parallel, then link the library."""
    from concurrent.futures import ThreadPoolExecutor

    import tempfile

    inc = ["-I", os.path.join(ROOT, "include")]
    cflags = [f for f in HIPCC_FLAGS if f != "-shared"] + inc + ["-c"]
    with tempfile.TemporaryDirectory(prefix="mplb_build_") as tmp:
        objs = [os.path.join(tmp, os.path.splitext(s)[0] + ".o") for s in SOURCES]
        with ThreadPoolExecutor(len(SOURCES)) as ex:
            jobs = [ex.submit(_compile, cflags + ["-x", "hip", os.path.join(CSRC, s)], o, verbose)
                    for s, o in zip(SOURCES, objs)]
            for j in jobs:
                j.result()
        _compile(["--offload-arch=gfx950", "-shared", "-fPIC", "--hip-link"] + objs, LIB, verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
