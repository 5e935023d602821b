"""Build the gfx950 shared library libnqs.so in-tree with hipcc.

Every source is compiled for gfx950 only, with packed FP32 instructions
disabled, and linked into ``paper_2206_14307_amd/libnqs.so``.  Objects go to
``_build/`` next to this file.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
OUT = os.path.join(HERE, "libnqs.so")
BUILD = os.path.join(HERE, "_build")
SOURCES = ["api.cpp", "tables.cpp", "lds_layout.cpp", "k_prep.hip", "k_theta.hip", "k_eloc.hip", "k_eloc_reg.hip", "k_eloc_fused.hip", "k_eloc_wide.hip", "k_grad.hip", "k_grad_fused.hip", "k_grad_wide.hip",
           "k_sample.hip", "k_sr.hip", "k_enum.hip", "k_sq.hip", "k_vmc.hip", "k_cg.hip",
           "k_lanczos2.hip", "k_noalloc.hip"]
ARCH = "gfx950"


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP toolchain is required to build libnqs.so")


def _flags(src):
    common = ["-O3", "-std=c++17", "-fPIC", f"-I{INCLUDE}", f"-I{CSRC}", "-Wall",
              "-Wno-unused-result"]
    if src.endswith(".hip"):
        return common + [f"--offload-arch={ARCH}", "-x", "hip",
                         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                         "-munsafe-fp-atomics",
                         # MFMA accumulators in ordinary VGPRs: the epilogues read every
                         # result, and AGPR accumulators cost a copy per register
                         "-mllvm", "-amdgpu-mfma-vgpr-form"]
    return common + ["-D__HIP_PLATFORM_AMD__"]


def _compile(src):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc()] + _flags(src) + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj, r.stderr


def build(verbose=False, jobs=None):
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 1)
    with cf.ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(_compile, SOURCES))
    objs = [o for o, _ in results]
    if verbose:
        for (o, err) in results:
            msgs = [l for l in err.splitlines() if "packed-fp32-ops" not in l]
            if msgs:
                print("\n".join(msgs), file=sys.stderr)
    tmp = OUT + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"linking failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
