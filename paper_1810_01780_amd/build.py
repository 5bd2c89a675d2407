"""Build the HIP library in-tree (gfx950 only)."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libradiotrace.so")
OBJDIR = os.path.join(ROOT, "_build")
SOURCES = ["rt_kernels.hip", "rt_mlp.hip", "rt_surrogate.hip", "rt_probe.hip", "rt_host.cpp"]
# Sources compiled with extra code-generation flags: the stratified trace
# kernel and the shot kernels keep constant materialisations in their step
# loops (no machine-level loop-invariant hoisting), which frees the
# registers they would hold (shot kernels: 129-141 VGPRs and no spills,
# against 168 VGPRs and 56-87 spilled with hoisting); the general trace
# kernel measured slower with the same flag.
SEPARATE = {"rt_strat.hip": ["-mllvm", "-disable-machine-licm"],
            "rt_solve.hip": ["-mllvm", "-disable-machine-licm"]}

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.isabs(cand) and os.path.exists(cand) or not os.path.isabs(cand)):
            return cand
    return "hipcc"


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stderr)


def build(verbose: bool = False) -> str:
    """Compile libradiotrace.so next to this file; always recompiles (every
    source to an object, in parallel, then one link)."""
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(OBJDIR, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include")]
    jobs = [(src, []) for src in SOURCES] + list(SEPARATE.items())
    objs = [os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o") for src, _ in jobs]
    cmds = [[hipcc(), *HIPCC_FLAGS, *extra, *inc, "-c", "-o", obj, os.path.join(CSRC, src)]
            for (src, extra), obj in zip(jobs, objs)]
    with ThreadPoolExecutor(max_workers=min(len(cmds), os.cpu_count() or 1)) as ex:
        list(ex.map(lambda c: _run(c, verbose), cmds))
    # ROCTx (the rocprofiler-sdk marker library) for the host ranges
    _run([hipcc(), "--offload-arch=gfx950", "-fPIC", "-shared", "-o", LIB + ".tmp", *objs,
          "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib"], verbose)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
