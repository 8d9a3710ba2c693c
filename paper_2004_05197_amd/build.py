"""Compile the HIP library libcellfft.so for gfx950 (in-tree).

Usage: python -m paper_2004_05197_amd.build   (or build() from Python)
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libcellfft.so")
SOURCES = ["fft.hip", "stencil.hip", "hyper.hip", "surrogate.hip", "solver.hip", "capi.hip", "noalloc.hip", "strainproj.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17",
    # packed FP32 instructions are not generated (see the design notes)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    "-Wno-unused-result",
]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed: " + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    return r


def build(verbose=False):
    os.makedirs(OBJ, exist_ok=True)
    objs = []
    cmds = []
    for src in SOURCES:
        obj = os.path.join(OBJ, src.replace(".hip", ".o"))
        objs.append(obj)
        cmds.append([HIPCC] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj])
    with ThreadPoolExecutor(max_workers=len(cmds)) as ex:
        for r in ex.map(_run, cmds):
            if verbose and (r.stdout or r.stderr):
                print(r.stdout + r.stderr)
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    return LIB


# Host-sanitized variant for the CPU tests of the C ABI: the host code (argument
# checks, handle bookkeeping, schedule cache, error paths) built with
# AddressSanitizer and UndefinedBehaviorSanitizer; the device code is
# unchanged.  The library loads into a Python started with the clang ASan
# runtime preloaded (see tests/test_abi_sanitized.py).
SAN_OBJ = os.path.join(HERE, "_build_asan")
SAN_LIB = os.path.join(SAN_OBJ, "libcellfft_asan.so")
CLANGXX = os.environ.get("CLANGXX", "/opt/rocm/lib/llvm/bin/clang++")
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g"]


def sanitizer_runtime():
    r = _run([CLANGXX, "-print-file-name=libclang_rt.asan-x86_64.so"])
    return r.stdout.strip()


def build_sanitized(verbose=False):
    os.makedirs(SAN_OBJ, exist_ok=True)
    objs, cmds = [], []
    for src in SOURCES:
        obj = os.path.join(SAN_OBJ, src.replace(".hip", ".o"))
        objs.append(obj)
        cmds.append([HIPCC] + FLAGS + SAN_FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj])
    with ThreadPoolExecutor(max_workers=len(cmds)) as ex:
        for r in ex.map(_run, cmds):
            if verbose and (r.stdout or r.stderr):
                print(r.stdout + r.stderr)
    # the objects carry their device code; the link is a host link against
    # the HIP runtime and the shared sanitizer runtime
    tmp = SAN_LIB + ".tmp"
    san = ",".join(["address", "undefined"])
    _run([CLANGXX, "-shared", "-fPIC", "-shared-libsan", "-fsanitize=" + san, "-o", tmp] + objs +
         ["-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"])
    os.replace(tmp, SAN_LIB)
    return SAN_LIB


# Bounds-checked variant for the debug tests: the kernels compare their field,
# spectrum, material and partial-sum accesses with the buffer extents and
# count (and skip) the ones out of range (cell_debug_bounds_violations()).
CHK_OBJ = os.path.join(HERE, "_build_checked")
CHK_LIB = os.path.join(CHK_OBJ, "libcellfft_checked.so")


def build_checked(verbose=False):
    os.makedirs(CHK_OBJ, exist_ok=True)
    objs, cmds = [], []
    for src in SOURCES:
        obj = os.path.join(CHK_OBJ, src.replace(".hip", ".o"))
        objs.append(obj)
        cmds.append([HIPCC] + FLAGS + ["-DCELLFFT_BOUNDS_CHECK", "-c", os.path.join(CSRC, src), "-o", obj])
    with ThreadPoolExecutor(max_workers=len(cmds)) as ex:
        for r in ex.map(_run, cmds):
            if verbose and (r.stdout or r.stderr):
                print(r.stdout + r.stderr)
    tmp = CHK_LIB + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, CHK_LIB)
    return CHK_LIB


if __name__ == "__main__":
    if "--checked" in sys.argv:
        print(build_checked(verbose="-v" in sys.argv))
    elif "--sanitize" in sys.argv:
        print(build_sanitized(verbose="-v" in sys.argv))
    else:
        print(build(verbose="-v" in sys.argv))
