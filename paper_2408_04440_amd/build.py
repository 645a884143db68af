"""Build libmpchol.so (HIP for gfx950) in-tree with hipcc.

Every library source under csrc/ is compiled to an object in _build/ (in
parallel) and linked into paper_2408_04440_amd/libmpchol.so.  The MFMA
throughput tool csrc/mfma_peak.hip is built beside it as the executable
paper_2408_04440_amd/mfma_peak.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libmpchol.so")
PEAK_OUT = os.path.join(HERE, "mfma_peak")
BUILD = os.path.join(ROOT, "_build")

ARCH = os.environ.get("MPCHOL_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# Packed FP32 instructions are turned off for all device code.  MFMA
# accumulators live in ordinary VGPRs (-amdgpu-mfma-vgpr-form): otherwise
# kernels of 256 threads keep them in AGPRs and copy them to and from VGPRs
# inside their K loops, each copy waiting for the MFMA that wrote it.
FLAGS = ["-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang",
         "-packed-fp32-ops", "-mllvm", "-amdgpu-mfma-vgpr-form", "-I", os.path.join(ROOT, "include"),
         "-Wno-unused-result"]

SOURCES = ["k_tiles.hip", "k_factor.hip", "k_ozaki.hip", "k_residual.hip", "k_estimate.hip", "k_apply.hip",
           "k_mlp.hip", "k_samples.hip", "k_sht.hip", "mpchol.cpp"]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC, *FLAGS, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def _build_peak_tool() -> str:
    tmp = PEAK_OUT + ".tmp"
    cmd = [HIPCC, *FLAGS, "-x", "hip", os.path.join(CSRC, "mfma_peak.hip"), "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for mfma_peak.hip:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, PEAK_OUT)
    return PEAK_OUT


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES) + 1)) as ex:
        tool = ex.submit(_build_peak_tool)
        objs = list(ex.map(_compile, SOURCES))
        tool.result()
    tmp = OUT + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
