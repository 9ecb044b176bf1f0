"""Builds the HIP library ``libmda.so`` for gfx950 in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libmda.so")
BUILD_DIR = os.path.join(HERE, "_build")

SOURCES = (["mda_wave_ns%d.hip" % t for t in (64, 56, 52, 48, 40)] + ["mda_group_ns%d.hip" % t for t in (64, 56, 48, 40)]
           + ["mda_wave_ns%d.hip" % t for t in (32, 28, 24, 16, 8)] + ["mda_group_ns%d.hip" % t for t in (32, 24, 16, 8)]
           + ["mda_wave64_ns%d.hip" % t for t in (64, 56, 52, 48, 40, 32, 28, 24, 16, 8)]
           + ["mda_generic_k%d.hip" % k for k in (4, 3, 2, 1)] + ["mda_generic_host.cpp"]
           + ["mda_kernels.hip", "mda_group.hip", "mda_front.hip", "mda_host.cpp", "mda_server.cpp"])

HIPCC = os.environ.get("HIPCC", "hipcc")
ARCH = os.environ.get("MDA_OFFLOAD_ARCH", "gfx950")

COMMON = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-ffp-contract=off", "-Wall", "-Wno-unused-result",
    "-I" + INCLUDE, "-I" + CSRC,
]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *COMMON, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed on " + src)
    return obj


def build(verbose: bool = False) -> str:
    """Compiles every source and links ``libmda.so`` (always rebuilds)."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    workers = max(1, min(len(SOURCES), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp, *objs]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("link failed")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
