"""Compile the HIP sources into the in-tree shared library ``liblbp.so`` (gfx950)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbp.so")
SOURCES = ["runtime.hip", "server.hip", "plan.hip", "bp_kernel.hip", "bp_int8_kernel.hip", "osd_kernel.hip",
           "baseline.hip"]
ARCH = os.environ.get("LBP_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


# The OSD kernels take LDS atomics from one lane that a data-dependent test picked;
# the compiler's atomic optimizer would wrap each in a lane election it cannot drop.
EXTRA_FLAGS = {"osd_kernel.hip": ["-mllvm", "-amdgpu-atomic-optimizer-strategy=None"]}


def build(verbose: bool = False) -> str:
    """Always recompiles (objects in parallel), then links liblbp.so atomically."""
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, src.replace(".hip", ".o"))
        cmd = [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall",
               "-mcode-object-version=5",
               # keep the compiler from forming packed-fp32 VALU instructions
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-c", os.path.join(CSRC, src), "-o", obj] + EXTRA_FLAGS.get(src, [])
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT))
        objs.append(obj)
    failed = False
    for p, src in zip(procs, SOURCES):
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        text = "\n".join(l for l in text.splitlines() if "packed-fp32-ops" not in l and l.strip())
        if p.returncode != 0:
            failed = True
            sys.stderr.write(f"--- {src}\n{text}\n")
        elif verbose and text:
            print(text)
    if failed:
        raise RuntimeError("hipcc failed")
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-mcode-object-version=5", "-shared", "-fPIC", "-o", tmp] + objs
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
