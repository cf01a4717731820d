"""Build the HIP library libsc.so for gfx950 with hipcc (in-tree).

Every .hip file under csrc/ is compiled to an object in _build/ and linked
into paper_2605_30396_amd/libsc.so.  Packed FP32 instructions are disabled for
all device code.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libsc.so")
ARCH = "gfx950"

CXXFLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-fPIC",
    "-std=c++17",
    "-Wno-unused-result",
    "-Wno-unused-value",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # the pursuit's step loop is unrolled over the sparsity cap so that its
    # per-step arrays stay in registers; at caps 24 and 32 the body exceeds
    # the default size limit of a forced unroll
    "-mllvm", "-pragma-unroll-threshold=200000",
]


# Kernels whose MFMA accumulators live only through the correlation stage:
# VGPR-form MFMA lets the pursuit reuse those registers (accumulation
# registers would stay allocated for the whole kernel and cost a wave per SIMD).
EXTRA = {
    "omp_batch_mfma.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
    "omp_batch_bf16.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
    "omp_multi.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
    "omp_csc_mfma.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
    "omp_csc_bf16.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
}


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src)[:-4] + ".o")
    cmd = ["hipcc", *CXXFLAGS, *EXTRA.get(os.path.basename(src), []), "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    # the host pass does not know the GPU feature flag; that warning is expected
    err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{err}")
    if err.strip():
        sys.stderr.write(err + "\n")
    return obj


def build(jobs: int | None = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(len(srcs), max(1, len(os.sched_getaffinity(0))))
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    r = subprocess.run(["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
