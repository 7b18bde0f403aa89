"""Build the HIP/C++ library libamg.so for gfx950 in-tree.

Usage: python -m paper_2202_11288_amd.build   (or build() from Python)
       python -m paper_2202_11288_amd.build --sanitize   (host-sanitizer build)
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libamg.so")
BUILD_DIR = os.path.join(ROOT, "_build")

SOURCES = [("fourstep_f64.hip", True), ("fourstep_f32.hip", True), ("amg_kernels.hip", True),
           ("amg_setup.hip", True), ("amg_api.cpp", True), ("amg_host.cpp", False)]

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          "-I" + os.path.join(ROOT, "include")]
# gfx950 only; packed FP32 instructions are disabled for every device pass.
DEVICE = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-command-line-argument"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libamg.so)")


# The host-sanitizer build: the host sources (the ABI, request server and
# allocator; the host numerics) with AddressSanitizer and UndefinedBehavior-
# Sanitizer on their host pass only, linked with the device objects of the
# plain build.  Output outside the package (it is not the product library);
# loaded through AMG_LIBRARY with the sanitizer runtime preloaded.
SAN_DIR = os.path.join(BUILD_DIR, "san")
SAN_LIB = os.path.join(SAN_DIR, "libamg_asan.so")
SAN_SOURCES = ("amg_api.cpp", "amg_host.cpp")
SAN_FLAGS = ("-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined "
             "-Xarch_host -fno-sanitize-recover=undefined "
             "-Xarch_host -fno-omit-frame-pointer -g").split()


def _compile(src: str, hip: bool, san: bool = False) -> str:
    out_dir = SAN_DIR if san else BUILD_DIR
    os.makedirs(out_dir, exist_ok=True)
    obj = os.path.join(out_dir, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc()] + COMMON + (["-x", "hip"] + DEVICE if hip else []) + \
        (SAN_FLAGS if san else []) + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda s: _compile(*s), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


def sanitizer_runtime() -> str:
    """The compiler's AddressSanitizer runtime (to preload)."""
    import glob
    root = os.path.dirname(os.path.dirname(os.path.realpath(hipcc())))
    hits = sorted(glob.glob(os.path.join(root, "llvm", "lib", "clang", "*", "lib", "linux",
                                         "libclang_rt.asan-x86_64.so")))
    if not hits:
        raise RuntimeError("the AddressSanitizer runtime of hipcc's clang was not found")
    return hits[-1]


def build_sanitized(verbose: bool = False) -> str:
    """The host-sanitizer library (plain device objects + instrumented host
    sources); the plain objects are built first if they are missing."""
    plain = {}
    for src, hip in SOURCES:
        obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
        plain[src] = (obj, hip)
    # plain objects older than any source or header are rebuilt
    newest = max(os.path.getmtime(os.path.join(d, f))
                 for d in (CSRC, os.path.join(ROOT, "include")) for f in os.listdir(d))
    missing = [(src, hip) for src, (obj, hip) in plain.items()
               if src not in SAN_SOURCES and
               (not os.path.exists(obj) or os.path.getmtime(obj) < newest)]
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        list(ex.map(lambda sh: _compile(*sh), missing))
        san = list(ex.map(lambda src: _compile(src, dict(SOURCES)[src], True), SAN_SOURCES))
    objs = [plain[src][0] for src, _ in SOURCES if src not in SAN_SOURCES] + san
    tmp = SAN_LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-shared-libasan"] + \
        SAN_FLAGS + ["-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, SAN_LIB)
    if verbose:
        print("built", SAN_LIB)
    return SAN_LIB


if __name__ == "__main__":
    if "--sanitize" in sys.argv[1:]:
        build_sanitized(verbose=True)
    else:
        build(verbose=True)
    sys.exit(0)
