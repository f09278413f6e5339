"""Build libnuhalo.so (HIP for gfx950) in-tree.

Every source is compiled with hipcc for gfx950 only.  Packed-FP32 VALU
instructions are disabled for all device code.  Run as a script or through
``__graft_entry__.build()``; it always recompiles.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libnuhalo.so")

SOURCES = [
    "host_physics.cpp",
    "host_api.cpp",
    "host_batch.cpp",
    "host_serve.cpp",
    "host_tune.cpp",
    "kernels_f64.hip",
    "kernels_f32c.hip",
    "kernels_batch.hip",
    "noalloc.hip",
    "device_fn.hip",
]

ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def common_flags():
    return [
        f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        # three-operand v_fma_f64 instead of the two-address v_fmac_f64: the
        # latter forces a v_mov pair for every FP64 constant addend (Horner steps)
        "-Xclang", "-target-feature", "-Xclang", "-fmacf64-inst",
        "-Wall", "-Wno-unused-command-line-argument",
        # fuse a*b+c only within one source expression: the same per-trajectory
        # code then rounds identically in the plain and the batched kernels
        "-ffp-contract=on",
        # keep loop-invariant FP64 constants out of the register file: hoisting
        # them out of the trajectory loops costs more registers than it saves
        "-mllvm", "-disable-machine-licm",
        "-I", INCLUDE, "-I", CSRC,
    ]


def build(verbose: bool = False, jobs: int = 8) -> str:
    cc = hipcc()
    tmp = tempfile.mkdtemp(prefix="nuhalo_build_")
    try:
        objs, procs = [], []
        for src in SOURCES:
            path = os.path.join(CSRC, src)
            obj = os.path.join(tmp, os.path.splitext(src)[0] + ".o")
            lang = ["-x", "hip"]
            cmd = [cc, *common_flags(), *lang, "-c", path, "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
            objs.append(obj)
            while sum(p.poll() is None for _, p in procs) >= jobs:
                procs[0][1].wait()
        failed = []
        for src, p in procs:
            out, _ = p.communicate()
            text = out.decode(errors="replace")
            if p.returncode != 0:
                failed.append((src, text))
            elif verbose and text.strip():
                print(text)
        if failed:
            msg = "\n".join(f"--- {s}\n{t}" for s, t in failed)
            raise RuntimeError(f"hipcc failed:\n{msg}")
        out_tmp = LIB + ".tmp"
        link = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", out_tmp, *objs,
                "-Wl,-rpath,/opt/rocm/lib"]
        if verbose:
            print(" ".join(link), flush=True)
        subprocess.run(link, check=True)
        os.replace(out_tmp, LIB)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
