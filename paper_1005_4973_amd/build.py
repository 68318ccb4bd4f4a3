"""Build libmtgp.so (HIP kernels for gfx950 + C ABI) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB_PATH = os.path.join(HERE, "libmtgp.so")
SOURCES = [os.path.join(CSRC, "mtgp_kernels.hip"), os.path.join(CSRC, "mtgp_api.cpp"),
           os.path.join(CSRC, "mtgp_f2.cpp"), os.path.join(CSRC, "mtgp_dc.cpp"), os.path.join(CSRC, "mtgp_serve.cpp"),
           os.path.join(CSRC, "mtgp_equidist.cpp")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-Wall",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
    "-pthread",
]


# the store-only probe that the benchmark times beside the generation kernels
# (a measurement aid, not part of the library)
PROBE_PATH = os.path.join(HERE, "libmtgp_probe.so")
PROBE_SOURCES = [os.path.join(CSRC, "store_probe.hip")]


def _compile(sources, path, verbose):
    tmp = path + ".tmp"
    cmd = [HIPCC] + FLAGS + ["-o", tmp] + sources
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed building {os.path.basename(path)}")
    os.replace(tmp, path)


def build(verbose: bool = False) -> str:
    _compile(SOURCES, LIB_PATH, verbose)
    _compile(PROBE_SOURCES, PROBE_PATH, verbose)
    return LIB_PATH


if __name__ == "__main__":
    print(build(verbose=True))
