"""Build the HIP library (libbemfmm.so) for gfx950 with hipcc, in-tree.

Every source is compiled to an object under _build/ and linked into
paper_1007_4591_amd/libbemfmm.so.  `build()` always recompiles (it is the
"does it build" check); `ensure_built()` builds only when the library is
missing or older than a source.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libbemfmm.so")
SOURCES = ["alloc.cpp", "tables.cpp", "tree_build.hip", "fmm.hip", "solve.hip", "yukawa.hip", "capi.cpp"]
ARCH = os.environ.get("BEMFMM_ARCH", "gfx950")


def _hipcc() -> str:
    for c in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"), shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _flags(src: str):
    f = ["-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}", "-Wall", "-Wno-unused-function",
         "-Wno-unused-variable", "-Wno-unused-but-set-variable", "-I", os.path.join(HERE, "..", "include")]
    if src.endswith(".hip"):
        # no packed FP32 VALU instructions in device code
        f += ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
    else:
        f += ["-x", "hip"]
    return f


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [_hipcc(), *_flags(src), "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(len(SOURCES), int(os.environ.get("MAX_JOBS", "8")))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


def ensure_built() -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES] + [os.path.join(CSRC, "common.h"),
                                                     os.path.join(HERE, "..", "include", "bemfmm.h")]
    if os.path.exists(LIB) and all(os.path.getmtime(LIB) >= os.path.getmtime(s) for s in srcs):
        return LIB
    return build()


if __name__ == "__main__":
    build(verbose=True)
