"""Build the HIP library libbp4.so for gfx950 in-tree (hipcc, no JIT cache).

Usage: python -m paper_2407_11523_amd.build
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libbp4.so")
ARCH = "gfx950"

SOURCES = ["bp4_api.cpp", "bp4_walk.cpp", "bp4_decode.hip", "bp4_sample.hip", "bp4_plain.hip", "bp4_soa.hip",
           "bp4_unrolled.hip", "bp4_noalloc.hip", "bp4_gather.hip"]

# Packed FP32 VALU forms are kept out of generated code.
HIP_FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-Wall",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return "hipcc"


def _compile(src: str) -> str:
    path = os.path.join(CSRC, src)
    obj = os.path.join(BUILD, src + ".o")
    cmd = [hipcc(), "-c", path, "-o", obj] + HIP_FLAGS
    if src.endswith(".hip"):
        cmd[1:1] = ["-x", "hip"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    """Compile every source and link libbp4.so; always rebuilds."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    _build_calibration()
    if verbose:
        print("built", LIB)
    return LIB


SAN_LIB = os.path.join(PKG, "libbp4_san.so")
# host code of the ABI layer only: the device code objects are the regular ones
HOST_SOURCES = ("bp4_api.cpp", "bp4_walk.cpp")
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined", "-g"]


def build_sanitized() -> str:
    """libbp4_san.so: the host sources bp4_api.cpp (argument checks, graph construction,
    launch set-up) and bp4_walk.cpp (walk order of the single-pass kernel) with
    AddressSanitizer and UndefinedBehaviorSanitizer, linked with the regular kernel
    objects; loaded with BP4_SANITIZE=1 and clang's ASan runtime preloaded."""
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    for src in SOURCES:
        if src in HOST_SOURCES:
            obj = os.path.join(BUILD, src.replace(".cpp", "_san.o"))
            cmd = [hipcc(), "-c", os.path.join(CSRC, src), "-o", obj] + HIP_FLAGS + SAN_FLAGS
            r = subprocess.run(cmd, capture_output=True, text=True)
            if r.returncode != 0:
                raise RuntimeError(f"hipcc failed for the sanitized {src}:\n{r.stdout}\n{r.stderr}")
            objs.append(obj)
        else:
            obj = os.path.join(BUILD, src + ".o")
            if not os.path.exists(obj):
                _compile(src)
            objs.append(obj)
    tmp = SAN_LIB + ".tmp"
    r = subprocess.run([hipcc(), "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs,
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed for the sanitized library:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, SAN_LIB)
    return SAN_LIB


def asan_runtime() -> str:
    """clang's ASan runtime of the ROCm toolchain (preloaded for the sanitized library)."""
    import glob
    cands = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not cands:
        raise RuntimeError("no libclang_rt.asan-x86_64.so under /opt/rocm/llvm")
    return cands[-1]


CALIB_SRC = os.path.join(PKG, "calib", "valu_rate.hip")
CALIB_BIN = os.path.join(PKG, "calib", "valu_rate")


def _build_calibration() -> None:
    """The VALU issue-rate calibration program (measures the roofline's peaks)."""
    cmd = [hipcc(), "-x", "hip", CALIB_SRC, "-o", CALIB_BIN + ".tmp"] + HIP_FLAGS
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for the calibration program:\n{r.stdout}\n{r.stderr}")
    os.replace(CALIB_BIN + ".tmp", CALIB_BIN)


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
