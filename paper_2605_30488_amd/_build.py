"""Builds libds3.so (HIP for gfx950) in-tree with hipcc.

Every translation unit is compiled for gfx950 only, with packed-FP32 instruction selection disabled,
then linked into one shared library next to this file.
"""
from __future__ import annotations

import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libds3.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["capi.cpp", "capi_match.cpp", "gn.hip", "chol.hip", "match.hip", "gauge.hip", "misc.hip",
           "adjoint.hip", "fuse.hip", "track.hip", "depth.hip", "spchol.hip", "tilechol.hip"]

FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-munsafe-fp-atomics",
         "-I", os.path.join(os.path.dirname(HERE), "include")]


# Per-source flags. chol.hip, tilechol.hip: matrix-core products read and write ordinary VGPRs instead of the
# accumulation registers, which removes a copy of every accumulator tile to and from them around each
# product in the diagonal factorisation's dependent chain.
# depth.hip: no contraction of float64 products and sums into fused multiply-adds, so that the segmentation
# features round exactly as the operations are written.
EXTRA = {"chol.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form=1"], "tilechol.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form=1"],
         "depth.hip": ["-ffp-contract=off"]}


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, *EXTRA.get(src, []), "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(jobs: int | None = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 4)
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
