"""Build libcgp.so (the gfx950 HIP kernels and the C-ABI runtime) in-tree.

    python -m paper_1308_3290_amd.build

Every call recompiles.  Objects go to paper_1308_3290_amd/_build/, the shared
library to paper_1308_3290_amd/libcgp.so.  The same call builds the
measurement library paper_1308_3290_amd/libcgp_stamps.so: the sources that
hold pass B, the fused one-layer stage pass and the C ABI compiled once more
with CGP_PHASE_STAMPS (phase stamps and cgp_phase_stamps), linked with the
other objects of libcgp.so.
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
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libcgp.so")
STAMPS_LIB = os.path.join(PKG, "libcgp_stamps.so")
SOURCES = ["solve_kernels.hip", "stencil_kernels.hip", "fused_kernels.hip", "fused2_kernels.hip",
           "adjoint_kernels.hip", "mg_kernels.hip", "persistent_kernels.hip", "runtime.hip"]
# sources compiled a second time, with the phase stamps, for libcgp_stamps.so
STAMPED = ["solve_kernels.hip", "fused_kernels.hip", "runtime.hip"]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm toolchain required to build libcgp.so)")


def compile_flags():
    return ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
            # no packed FP32 instructions in device code
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            # multiply-adds are fused only within one source expression, so
            # that the same expression rounds the same way in every kernel it
            # is inlined into (the fused pass and pass A must agree bit for bit)
            "-ffp-contract=on",
            # the first kernel arguments arrive preloaded in SGPRs (gfx940+),
            # which saves a dependent scalar load at the start of every
            # launch, ahead of the member descriptor's (about 1 us per step)
            "-mllvm", "-amdgpu-kernarg-preload-count=16",
            "-I", os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-result"]


# Per-source flags on top of compile_flags(): the column solve and the
# unfused passes are scheduled for instruction-level parallelism (the
# 512x1024 CGP-factor-2 step measured 1.3 % faster; the fused-pass sources
# measured slower with it and keep the default scheduler).
EXTRA_FLAGS = {"solve_kernels.hip": ["-mllvm", "-amdgpu-sched-strategy=max-ilp"]}


def build(verbose: bool = False) -> str:
    os.makedirs(os.path.join(BUILD, "stamps"), exist_ok=True)
    cc = hipcc()

    def one(job):
        src, stamped = job
        obj = os.path.join(BUILD, "stamps" if stamped else "", src.replace(".hip", ".o"))
        cmd = [cc, *compile_flags(), *EXTRA_FLAGS.get(src, []),
               *(["-DCGP_PHASE_STAMPS"] if stamped else []), "-c", os.path.join(CSRC, src),
               "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
        if verbose and r.stderr.strip():
            print(r.stderr)
        return obj

    jobs = [(s, False) for s in SOURCES] + [(s, True) for s in STAMPED]
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(one, jobs))
    plain = objs[:len(SOURCES)]
    stamped = dict(zip(STAMPED, objs[len(SOURCES):]))
    with_stamps = [stamped.get(s, o) for s, o in zip(SOURCES, plain)]
    for objects, lib in ((plain, LIB), (with_stamps, STAMPS_LIB)):
        tmp = lib + ".tmp"
        cmd = [cc, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objects, "-o", tmp]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
        os.replace(tmp, lib)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
