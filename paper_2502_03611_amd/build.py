"""Build libqn.so (HIP kernels + C ABI) for gfx950 in-tree with hipcc.

Each source is compiled to an object file by its own hipcc process (in
parallel), then the objects are linked into one shared library.

Usage: python -m paper_2502_03611_amd.build  (or build() from Python).
"""

import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libqn.so")

SOURCES = ["qn_gemm_fold.hip", "qn_gemm_bf16.hip", "qn_pointwise.hip", "qn_sem.hip", "qn_probe.hip",
           "qn_api.cpp", "qnn.hip", "qnn_api.cpp", "qn_batched.cpp"]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # keep packed-FP32 VALU instructions out of the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result", "-Wno-unused-function",
]


def hipcc():
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found: the ROCm toolchain is required to build libqn")
    return path


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed: " + " ".join(cmd[-3:]))


def build(verbose=False, jobs=None):
    """Compile every HIP source of the library into paper_2502_03611_amd/libqn.so."""
    cc = hipcc()
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    jobs = jobs or min(len(SOURCES), max(1, min(16, os.cpu_count() or 1)))
    with tempfile.TemporaryDirectory(prefix="qnbuild_") as tmpdir:
        objs, cmds = [], []
        for s in SOURCES:
            obj = os.path.join(tmpdir, s + ".o")
            objs.append(obj)
            cmds.append([cc] + FLAGS + inc + ["-c", os.path.join(CSRC, s), "-o", obj])
        with ThreadPoolExecutor(max_workers=jobs) as pool:
            for fut in [pool.submit(_run, c, verbose) for c in cmds]:
                fut.result()
        tmp = LIB + ".tmp"
        _run([cc, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", tmp], verbose)
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
