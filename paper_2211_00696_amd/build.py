"""Build the C-ABI shared library libphiq.so for gfx950 with hipcc (in-tree)."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libphiq.so")

SOURCES = ["kernels.hip", "kernels_slab.hip", "kernels_lowp.hip", "kernels_bf16r.hip", "kernels_f32r.hip", "kernels_f64r.hip", "kernels_i8.hip", "batched.hip", "etd.hip", "exprk.hip", "mlp.hip", "noalloc.hip", "planner.cpp", "plan.cpp", "launch.cpp", "gauss.cpp", "int8.cpp", "combo.cpp", "cc.cpp", "autotune.cpp", "api.cpp", "batched.cpp",
           "etd.cpp", "exprk.cpp", "mlp.cpp"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-Wall",
    "-Wno-unused-result",
    # keep the compiler from forming packed FP32 instructions (they are not
    # trusted on this target)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return "hipcc"


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
    return res.returncode


def build(verbose: bool = False, jobs: int = 8) -> str:
    """Compile every source to an object in _build/ (in parallel), then link."""
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    objdir = os.path.join(ROOT, "_build")
    os.makedirs(objdir, exist_ok=True)
    compile_flags = [f for f in HIPCC_FLAGS if f != "-shared"]
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    objs = [os.path.join(objdir, s.replace(".", "_") + ".o") for s in srcs]
    cmds = [[hipcc(), *compile_flags, *inc, "-c", os.path.join(CSRC, s), "-o", o] for s, o in zip(srcs, objs)]
    with ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        codes = list(ex.map(lambda c: _run(c, verbose), cmds))
    if any(codes):
        raise RuntimeError("hipcc failed building libphiq.so")
    tmp = LIB + ".tmp"
    if _run([hipcc(), "--offload-arch=gfx950", "-fPIC", "-shared", *objs, "-o", tmp], verbose):
        raise RuntimeError("hipcc failed linking libphiq.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
