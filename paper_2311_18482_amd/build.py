"""Build liblegs.so (all HIP sources, gfx950) in-tree next to this file.

Flags:
  --offload-arch=gfx950         CDNA4 only
  -ffp-contract=off             every float operation is rounded as written, so
                                the forward and backward blend kernels evaluate
                                alpha with one identical instruction sequence and
                                the float64 projection decides boxes exactly
  -munsafe-fp-atomics           hardware global float atomics (no CAS loops)
  -Xclang -target-feature -Xclang -packed-fp32-ops
                                no packed FP32 instructions
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "liblegs.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-ffp-contract=off",
         "-munsafe-fp-atomics", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument", "-I", os.path.join(ROOT, "include"), "-I", CSRC]


# Per-source additions. The decoders keep MFMA accumulators in ordinary VGPRs
# (the VGPR form of the MFMA instructions that gfx950 has): their results are
# read by VALU code right away (ReLU and bf16 packing, the argmax), which from
# accumulation registers would cost one extra move per value.
EXTRA = {"decode.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
         "mlp.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
         "language.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
         "smooth.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def _compile(src, verbose):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC] + FLAGS + EXTRA.get(os.path.basename(src), []) + ["-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False, jobs: int = 4) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), srcs))
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", LIB + ".tmp"] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
