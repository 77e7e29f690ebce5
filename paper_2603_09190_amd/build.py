"""Build libzippir.so (HIP for gfx950) in-tree with hipcc.

Every source under csrc/ is compiled to an object in _build/ and linked into
paper_2603_09190_amd/libzippir.so.  Run as ``python -m paper_2603_09190_amd.build``.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libzippir.so")
ARCH = os.environ.get("ZIPPIR_ARCH", "gfx950")

SOURCES = ["runtime.cpp", "serve.cpp", "compressor.cpp", "matvec.hip", "gemm_i8.hip", "rows.hip", "hint.hip",
           "compress.hip", "offset.hip", "lwec.hip", "probe.hip", "answer.hip", "prg.hip", "noalloc.hip", "batch.hip", "hgemm.hip",
           "unpack.hip"]

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          "-I", os.path.join(ROOT, "include"), "-I", CSRC,
          "-Wall", "-Wno-unused-function"]
# no packed-fp32 instruction selection in device code
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# Contractions whose accumulators fit the architectural VGPRs: MFMA accumulators allocated there
# instead of in AGPRs, which keeps the register allocator from rotating them through copies
# between the MFMAs of the main loop.
MFMA_VGPR_FORM = ["-mllvm", "-amdgpu-mfma-vgpr-form"]
PER_FILE_FLAGS = {"offset.hip": MFMA_VGPR_FORM, "hgemm.hip": MFMA_VGPR_FORM, "batch.hip": MFMA_VGPR_FORM,
                  "unpack.hip": MFMA_VGPR_FORM}


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC, *COMMON, *DEVICE_FLAGS, *PER_FILE_FLAGS.get(src, []), "-x", "hip", "-c", os.path.join(CSRC, src),
           "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
