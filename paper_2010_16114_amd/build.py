"""Build libcoxhip.so (the HIP kernels and the C ABI) for gfx950, in-tree.

Each source is compiled to an object with hipcc in parallel, then linked into a
shared library next to this file.  Usage: ``python -m paper_2010_16114_amd.build``.
"""
from __future__ import annotations

import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libcoxhip.so")
SOURCES = ["api.cpp", "risk.hip", "gemv.hip", "gemvt.hip", "misc.hip", "mfma.hip", "covar.hip", "refit.hip", "nmf.hip",
           "persist.hip"]
ARCH = os.environ.get("COXHIP_ARCH", "gfx950")
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # packed FP32 instructions are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    "-Wall", "-Wno-unused-result",
]


# sources of the tuned matrix-core kernels: their hash keys the autotuner's cache
TUNED = ["mfma.hip", "mfma.h", "device_common.h"]


def source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in TUNED:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _compile(src: str) -> str:
    out = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
    cmd = ["hipcc", "-x", "hip", "-c", os.path.join(CSRC, src), "-o", out] + FLAGS
    if src == "api.cpp":
        cmd.append(f"-DCOXHIP_SRC_HASH=\"{source_hash()}\"")
    r = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    err = "\n".join(l for l in r.stderr.splitlines() if noise not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{err}")
    if err.strip():
        print(err, file=sys.stderr)
    return out


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    rocm_lib = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib")
    subprocess.run(["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs +
                   [f"-L{rocm_lib}", f"-Wl,-rpath,{rocm_lib}", "-lrocprofiler-sdk-roctx"], check=True)
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
