"""Build the R3MG-C HIP library (libr3mg.so) in-tree for gfx950 with hipcc.

Usage: python -m paper_2607_28235_amd.build   (or build() from the package root)
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libr3mg.so")
BUILD_DIR = os.path.join(HERE, "_build")

SOURCES = ["kernels.hip", "matfree.hip", "noalloc.hip", "solver.cpp", "capi.cpp", "analysis.cpp", "matfree.cpp",
           "tunecache.cpp"]

COMMON = ["-O3", "-std=c++17", "-fPIC", "-I", INCLUDE, "-I", CSRC, "--offload-arch=gfx950",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-result"]
PER_FILE = {
    # host decisions (tree comparisons, unisolvence pivots, transfer values) without FMA contraction
    "analysis.cpp": ["-ffp-contract=off"],
    "matfree.cpp": ["-ffp-contract=off"],
}


def _hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    return "hipcc"


def _compile(src: str) -> str:
    obj = os.path.join(BUILD_DIR, src + ".o")
    cmd = [_hipcc(), *COMMON, *PER_FILE.get(src, []), "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(4, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp, *objs, "-pthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


# Host-sanitized variant for testing the host code on the CPU: the analysis, the matrix-free set-up and the C ABI
# are compiled with AddressSanitizer and UndefinedBehaviorSanitizer on their host side only (device code is never
# sanitized), and linked with the ordinary objects of the other sources.  Load it with R3MG_LIBRARY pointing at it
# and the compiler's ASan runtime preloaded (sanitizer_runtime()).
SAN_LIB = os.path.join(HERE, "libr3mg_san.so")
SAN_DIR = os.path.join(HERE, "_build_san")
SAN_SOURCES = ["analysis.cpp", "matfree.cpp", "capi.cpp"]
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer", "-g"]


def sanitizer_runtime() -> str:
    """Path of the ASan runtime matching hipcc's compiler (to LD_PRELOAD into an unsanitized Python)."""
    r = subprocess.run([os.path.join(os.path.dirname(_hipcc()), "..", "llvm", "bin", "clang"),
                        "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    if r.returncode != 0 or not os.path.exists(path):
        raise RuntimeError("ASan runtime of the ROCm compiler not found")
    return path


def build_sanitized(verbose: bool = False) -> str:
    os.makedirs(SAN_DIR, exist_ok=True)
    objs = []
    for src in SOURCES:
        if src not in SAN_SOURCES:
            obj = os.path.join(BUILD_DIR, src + ".o")
            if not os.path.exists(obj):
                build()
            objs.append(obj)
            continue
        obj = os.path.join(SAN_DIR, src + ".o")
        cmd = [_hipcc(), *COMMON, *PER_FILE.get(src, []), *SAN_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
        objs.append(obj)
    # no sanitizer flags at the link: the sanitizer entry points stay undefined in the library and are resolved
    # from the runtime preloaded into the process (its ASan runtime carries the UBSan handlers as well)
    cmd = [_hipcc(), "-shared", "-fPIC", "--offload-arch=gfx950", "-o", SAN_LIB, *objs, "-pthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    if verbose:
        print("built", SAN_LIB)
    return SAN_LIB


if __name__ == "__main__":
    if "--sanitized" in sys.argv:
        build_sanitized(verbose=True)
    else:
        build(verbose=True)
    sys.exit(0)
