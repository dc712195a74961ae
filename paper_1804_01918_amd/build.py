"""Build libd2q37.so (all HIP sources under csrc/) for gfx950 with hipcc.

Run as ``python -m paper_1804_01918_amd.build`` or through
``__graft_entry__.build()``. The library is written next to this file so
that it travels with the source tree.
"""
from __future__ import annotations

import glob
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libd2q37.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
ARCH = os.environ.get("D2Q37_OFFLOAD_ARCH", "gfx950")

HIPFLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # Rounding is as written: fused multiply-adds only where the source
    # spells them, so kernels sharing device code round identically.
    "-ffp-contract=off",
    # No packed FP32 instructions in device code.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
    f"-I{INCLUDE}",
]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the D2Q37 library needs the ROCm toolchain")


def sources() -> list[str]:
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def build(verbose: bool = False, jobs: int = 4, defines=(), out: str | None = None) -> str:
    """Compile and link; `defines` are extra -D macros, `out` an alternative
    library path (the default is the package's libd2q37.so)."""
    hipcc = _hipcc()
    lib = out or LIB
    objdir = os.path.join(os.path.dirname(lib), "_build" if out is None else "_build_" + os.path.basename(lib))
    os.makedirs(objdir, exist_ok=True)

    def compile_one(src: str) -> str:
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        cmd = [hipcc, *HIPFLAGS, *[f"-D{d}" for d in defines], "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{res.stderr}")
        err = "\n".join(l for l in res.stderr.splitlines() if "packed-fp32-ops" not in l)
        if verbose and err.strip():
            print(err, file=sys.stderr)
        return obj

    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(compile_one, sources()))
    tmp = lib + f".tmp{os.getpid()}"
    cmd = [hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stderr}")
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("-v", action="store_true")
    ap.add_argument("-D", action="append", default=[], dest="defines")
    ap.add_argument("-o", default=None, dest="out")
    a = ap.parse_args()
    print(build(verbose=a.v, defines=a.defines, out=a.out))
