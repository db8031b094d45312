"""Builds libgmr.so (HIP, gfx950) in-tree with hipcc.

Every kernel source and the host API are compiled to objects and linked into
``paper_2602_14493_amd/libgmr.so``.  Flags:
  --offload-arch=gfx950      CDNA4 (MI355X) only
  -munsafe-fp-atomics        float atomics become hardware global_atomic_add_f32
  -ffp-contract=off          no implicit FMA contraction; the kernels write fmaf where they mean it,
                             so forward and backward take bit-identical alpha decisions
  -target-feature -packed-fp32-ops   no packed FP32 instructions are generated
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgmr.so")
SOURCES = ["k_project.hip", "k_bin.hip", "k_sort.hip", "k_raster.hip", "k_grad.hip", "k_recon.hip", "api.cpp"]
ARCH = "gfx950"


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found (ROCm is required to build libgmr)")


def flags() -> list[str]:
    return [f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17", "-munsafe-fp-atomics", "-ffp-contract=off",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wall", "-Wno-unused-command-line-argument",
            "-I" + os.path.join(HERE, "..", "include")]


def build(verbose: bool = False, jobs: int = 6) -> str:
    """Compile every source and link libgmr.so (always rebuilds)."""
    cc = hipcc()
    tmp = tempfile.mkdtemp(prefix="gmr_build_")
    try:
        def compile_one(src):
            obj = os.path.join(tmp, os.path.splitext(src)[0] + ".o")
            cmd = [cc, *flags(), "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
            r = subprocess.run(cmd, capture_output=True, text=True)
            if r.returncode != 0:
                raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
            if verbose and (r.stderr.strip()):
                print(r.stderr, file=sys.stderr)
            return obj

        with ThreadPoolExecutor(max_workers=jobs) as ex:
            objs = list(ex.map(compile_one, SOURCES))
        out_tmp = LIB + ".tmp"
        cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", out_tmp]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
        os.replace(out_tmp, LIB)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
