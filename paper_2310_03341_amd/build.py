"""Build libbdg.so (gfx950) in-tree from the HIP sources in csrc/.

Usage: python -m paper_2310_03341_amd.build   (or build() from Python)
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(os.path.dirname(HERE), "_build", "obj")
LIB = os.path.join(HERE, "libbdg.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Packed FP32 instructions are disabled on purpose: some of their forms have
# returned wrong results on gfx950 now and then, with no error raised.
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-result", "-I" + os.path.join(os.path.dirname(HERE), "include")]


# Per-file extra flags.  MFMA accumulators in ordinary VGPRs: the kernels here
# combine them with vector arithmetic, which AGPRs would need copies for.
EXTRA_FLAGS = {name: ["-mllvm", "-amdgpu-mfma-vgpr-form"]
               for name in ("bt2.hip", "gemm.hip", "he2hb.hip", "refine.hip")}
# The back-transformation-2 ring kernel unrolls its block loop by three; its
# product loops must still unroll fully (their tile and accumulator indices
# become constants, which keeps those arrays in registers), which needs a
# larger size limit for pragma-requested unrolling than the default.
EXTRA_FLAGS["bt2.hip"] = EXTRA_FLAGS["bt2.hip"] + ["-mllvm", "-pragma-unroll-threshold=1000000"]


def _compile(src: str) -> str:
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    cmd = [HIPCC] + HIP_FLAGS + EXTRA_FLAGS.get(os.path.basename(src), []) + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, r.stdout, r.stderr))
    return obj


def build(jobs: int | None = None) -> str:
    os.makedirs(OBJ, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    jobs = jobs or min(8, len(srcs))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (r.stdout, r.stderr))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(int(sys.argv[1]) if len(sys.argv) > 1 else None))
