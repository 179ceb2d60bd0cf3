"""Build the HIP library (gfx950) in-tree: paper_1602_06589_amd/libflapw_hip.so.

Every source under csrc/ is compiled by hipcc for gfx950 only, with packed-FP32 instruction
selection disabled, and linked into one shared library exporting the C-ABI of include/flapw.h.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OBJDIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libflapw_hip.so")
MFMA_RATE = os.path.join(HERE, "mfma_rate")                  # matrix-core ceiling microbenchmark
COPY_RATE = os.path.join(HERE, "copy_rate")                  # L2 -> LDS copy and LDS read rates
MOD_BLOCKS = os.path.join(HERE, "mod_blocks")                # block shapes of the modular contraction
ARCH = "gfx950"


def _hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))


FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-I", INCLUDE, "-I", CSRC,
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wall", "-Wno-unused-function",
         "-Wno-unused-command-line-argument"]


def _compile(src: str) -> str:
    obj = os.path.join(OBJDIR, os.path.basename(src) + ".o")
    cmd = [_hipcc()] + FLAGS + ["-c", src, "-o", obj]
    if src.endswith(".cpp"):
        cmd = [_hipcc()] + FLAGS + ["-x", "hip", "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{out}")
    if out.strip():
        sys.stderr.write(out + "\n")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    srcs = sources()
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp%d" % os.getpid()
    # rocSOLVER (and rocBLAS under it) for the dense generalized eigensolve
    cmd = [_hipcc(), "-shared", f"--offload-arch={ARCH}", "-o", tmp] + objs + [
        "-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lrocsolver", "-lrocblas"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    src = os.path.join(HERE, "microbench", "mfma_rate.hip")
    # VGPR-form MFMAs keep the register-only loops free of accumulator copies
    r = subprocess.run([_hipcc()] + [f for f in FLAGS if f != "-fPIC"] + ["-mllvm", "-amdgpu-mfma-vgpr-form=1", src,
                                                                          "-o", MFMA_RATE], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for mfma_rate.hip:\n" + r.stdout + r.stderr)
    src = os.path.join(HERE, "microbench", "copy_rate.hip")
    r = subprocess.run([_hipcc()] + [f for f in FLAGS if f != "-fPIC"] + [src, "-o", COPY_RATE], capture_output=True,
                       text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for copy_rate.hip:\n" + r.stdout + r.stderr)
    src = os.path.join(HERE, "microbench", "mod_blocks.hip")
    r = subprocess.run([_hipcc()] + [f for f in FLAGS if f != "-fPIC"] + [src, "-o", MOD_BLOCKS], capture_output=True,
                       text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for mod_blocks.hip:\n" + r.stdout + r.stderr)
    if verbose:
        print("built", LIB, MFMA_RATE, COPY_RATE, "and", MOD_BLOCKS)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
