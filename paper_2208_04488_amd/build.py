"""Build of the gfx950 library ``libhrm.so`` (hipcc, in-tree)."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libhrm.so")
SOURCES = ["hrm.hip", "hrm_batch.hip", "hrm_mlp.hip"]
# per-source flags: the persistent batch kernel wraps the face arithmetic in
# problem / step / stage / tile loops; machine-level loop-invariant code motion
# would lift dozens of FP64 constant materialisations out of them and keep
# them in vector registers for the whole launch (spills at two waves/SIMD)
SOURCE_FLAGS = {"hrm_batch.hip": ["-mllvm", "-disable-machine-licm"]}
ARCH = "gfx950"

# -packed-fp32-ops: the compiler emits no packed FP32 (v_pk_*_f32) instructions
HIPFLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False, extra=()) -> str:
    objs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, src + ".o")
        cmd = [hipcc(), *HIPFLAGS, *SOURCE_FLAGS.get(src, []), *extra, "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-c",
               os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB + ".tmp"
    subprocess.run([hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp], check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
