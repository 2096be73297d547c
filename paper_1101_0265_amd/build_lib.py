"""Build libsnf.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_1101_0265_amd.build_lib          # compile
    python -m paper_1101_0265_amd.build_lib --check  # compile, then check the exported symbols
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libsnf.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Packed-FP32 VALU ops are disabled for all device code (the compiler would otherwise form
# v_pk_* FP32 instructions from scalar / float2 code by itself).
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-mllvm", "-amdgpu-mfma-vgpr-form", "-Wno-unused-command-line-argument"]


def sources() -> list:
    return sorted(glob.glob(os.path.join(PKG, "csrc", "*.hip")))


def build(verbose: bool = False) -> str:
    """Compile every HIP source of the library into ``libsnf.so`` (always recompiles)."""
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, "-I", os.path.join(ROOT, "include"), "-o", tmp, *sources()]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed with exit code {r.returncode}")
    if verbose and r.stderr.strip():
        sys.stderr.write(r.stderr)
    os.replace(tmp, LIB)
    return LIB


def header_symbols() -> list:
    """Function names declared in include/*.h (the C ABI)."""
    import re
    names = []
    for h in sorted(glob.glob(os.path.join(ROOT, "include", "*.h"))):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*[A-Za-z_][\w\s\*]*?\b(snf_\w+)\s*\(", text, flags=re.M):
            names.append(m.group(1))
    return sorted(set(names))


if __name__ == "__main__":
    path = build(verbose=True)
    print("built", path)
    if "--check" in sys.argv:
        import ctypes
        lib = ctypes.CDLL(path)
        missing = [s for s in header_symbols() if not hasattr(lib, s)]
        print("declared:", header_symbols())
        if missing:
            raise SystemExit(f"missing exports: {missing}")
        print("all declared symbols exported")
