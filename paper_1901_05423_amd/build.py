"""Compile the HIP library in-tree for gfx950 (hipcc, no JIT cache)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librtforest.so")
SOURCES = ["rtf_abi.hip", "rtf_build.hip", "rtf_sample.hip", "rtf_quantize.hip",
           "rtf_backward.hip", "rtf_noalloc.hip", "rtf_alias.hip"]
# measurement aid: the sampling kernels' memory pattern without the search
PROBE_LIB = os.path.join(HERE, "librtf_probe.so")
PROBE_SOURCES = ["rtf_probe.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off",
    # no packed FP32 instructions anywhere
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
    "-I", os.path.join(ROOT, "include"),
]


def _link(out: str, sources, verbose: bool) -> str:
    tmp = out + ".tmp"
    cmd = [HIPCC, *FLAGS, "-o", tmp, *[os.path.join(CSRC, s) for s in sources]]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build_library(verbose: bool = False) -> str:
    """Build librtforest.so (and the measurement probe librtf_probe.so) from
    csrc/*.hip; returns the path of librtforest.so."""
    _link(PROBE_LIB, PROBE_SOURCES, verbose)
    return _link(LIB, SOURCES, verbose)


if __name__ == "__main__":
    print(build_library(verbose="-v" in sys.argv))
