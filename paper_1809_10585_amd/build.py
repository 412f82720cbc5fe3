"""Compile the HIP library libhodlr.so for gfx950 (in-tree, next to this file).

The kernels are split by family into translation units that compile in
parallel (csrc/k_*.hip), plus the host scheduler and C ABI (csrc/hodlr.cpp);
the objects are linked into one shared library.
"""
from __future__ import annotations

import concurrent.futures as cf
import hashlib
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
UNITS = ["hodlr.cpp", "check.cpp", "k_tr.hip", "k_mm.hip", "k_leaf.hip", "k_vec.hip"]
OUT = os.path.join(HERE, "libhodlr.so")
OBJ = os.path.join(ROOT, "_build")
ARCH = os.environ.get("HODLR_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _key(unit: str) -> str:
    """Content hash of a unit, every header of csrc/ and include/, and the flags."""
    h = hashlib.sha256(" ".join(FLAGS).encode())
    for d in (CSRC, os.path.join(ROOT, "include")):
        for f in sorted(os.listdir(d)):
            if f.endswith(".h") or f == unit:
                h.update(f.encode())
                h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def _compile(unit: str, reuse: bool) -> str:
    obj = os.path.join(OBJ, f"{unit}.{_key(unit)}.o")
    if reuse and os.path.exists(obj):
        return obj
    tmp = obj + ".tmp"
    cmd = [hipcc()] + FLAGS + ["-c", "-x", "hip", os.path.join(CSRC, unit), "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed for {unit}")
    os.replace(tmp, obj)
    return obj


def build(verbose: bool = False, reuse: bool | None = None) -> str:
    """Compile every unit (in parallel) and link libhodlr.so.  With reuse (or
    HODLR_BUILD_REUSE=1) an object whose sources and flags are unchanged is
    taken from _build/ instead of being compiled again."""
    if reuse is None:
        reuse = os.environ.get("HODLR_BUILD_REUSE") == "1"
    os.makedirs(OBJ, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=len(UNITS)) as ex:
        objs = list(ex.map(lambda u: _compile(u, reuse), UNITS))
    tmp = OUT + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC"] + objs + ["-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("linking libhodlr.so failed")
    if verbose:
        sys.stderr.write(r.stderr)
    os.replace(tmp, OUT)
    return OUT


# host-code sanitizer build: the scheduler, C ABI and hazard checker compiled
# with AddressSanitizer and UndefinedBehaviorSanitizer for the host side only
# (device code is not instrumented), linked with the regular kernel objects
ASAN_OUT = os.path.join(OBJ, "asan", "libhodlr.so")
HOST_UNITS = ["hodlr.cpp", "check.cpp"]
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]


def asan_runtime() -> str | None:
    base = "/opt/rocm/llvm/lib/clang"
    if not os.path.isdir(base):
        return None
    for ver in sorted(os.listdir(base), reverse=True):
        p = os.path.join(base, ver, "lib", "linux", "libclang_rt.asan-x86_64.so")
        if os.path.exists(p):
            return p
    return None


def build_asan() -> str:
    """libhodlr.so with the host units sanitized, in _build/asan/ (for the CPU
    tests of the C ABI; load it with the ASan runtime preloaded)."""
    os.makedirs(os.path.dirname(ASAN_OUT), exist_ok=True)
    kern = [_compile(u, True) for u in UNITS if u not in HOST_UNITS]
    objs = []
    for u in HOST_UNITS:
        obj = os.path.join(OBJ, "asan", f"{u}.{_key(u)}.o")
        if not os.path.exists(obj):
            cmd = [hipcc()] + FLAGS + ["-O1", "-g"] + SAN + ["-c", "-x", "hip", os.path.join(CSRC, u), "-o", obj]
            r = subprocess.run(cmd, capture_output=True, text=True)
            if r.returncode != 0:
                sys.stderr.write(r.stdout + r.stderr)
                raise RuntimeError(f"hipcc (sanitized) failed for {u}")
        objs.append(obj)
    cmd = ([hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-Xarch_host", "-shared-libasan"] + SAN
           + objs + kern + ["-o", ASAN_OUT])
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("linking the sanitized libhodlr.so failed")
    return ASAN_OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, reuse="--reuse" in sys.argv or None))
