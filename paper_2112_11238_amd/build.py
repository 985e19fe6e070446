"""Build libkp.so (the HIP C-ABI library) for gfx950 with hipcc, in-tree.

    python -m paper_2112_11238_amd.build          # compile and link
    python -m paper_2112_11238_amd.build --check  # compile only the host-side
                                                   # symbol check afterwards

Every .hip file under csrc/ is compiled to an object (in parallel) and the
objects are linked into paper_2112_11238_amd/libkp.so. The library links the
HIP runtime by its soname; the Python binding imports torch first, so the
process uses the one HIP runtime torch already loaded.
"""
from __future__ import annotations

import concurrent.futures
import hashlib
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libkp.so")
ARCH = "gfx950"

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-I", INCLUDE, "-I", CSRC,
    # packed FP32 vector ops stay off in all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
]


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm toolchain required to build libkp.so)")


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _compile(src):
    obj = os.path.join(BUILD, os.path.basename(src)[:-4] + ".o")
    cmd = [hipcc()] + HIPCC_FLAGS + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                     if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{msgs}")
    return obj, msgs


def build(verbose=True):
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    workers = min(len(srcs), int(os.environ.get("MAX_JOBS", "8")), 16)
    with concurrent.futures.ThreadPoolExecutor(max_workers=max(workers, 1)) as ex:
        results = list(ex.map(_compile, srcs))
    for obj, msgs in results:
        if msgs.strip() and verbose:
            print(msgs, file=sys.stderr)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + \
        [o for o, _ in results]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


# A build of the same sources with AddressSanitizer and
# UndefinedBehaviorSanitizer on the host code only (argument validation, the
# mode planner, workspace layouts, the batch plan, the tile table); the device
# code is compiled as usual, without instrumentation. It serves the host-side
# test suites, which never launch a kernel: load it by pointing KP_LIBRARY
# at it, with the clang ASan runtime preloaded.
HOSTSAN_LIB = os.path.join(BUILD, "hostsan", "libkp_hostsan.so")
HOSTSAN_FLAGS = [
    f"--offload-arch={ARCH}", "-O1", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE, "-I", CSRC,
    # the device code of this build is never launched: compile it unoptimised
    "-Xarch_device", "-O0",
    "-Xarch_host", "-g", "-Xarch_host", "-fno-omit-frame-pointer",
    "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
    "-Xarch_host", "-fno-sanitize-recover=undefined",
]


def _hostsan_stamp():
    h = hashlib.sha256(" ".join(HOSTSAN_FLAGS).encode())
    for src in sources() + sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                                  if f.endswith(".h")) + [os.path.join(INCLUDE, "kp.h")]:
        with open(src, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def asan_runtime():
    """The clang AddressSanitizer runtime matching hipcc's compiler."""
    import glob
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def build_hostsan(verbose=False, force=False):
    """Build (or, if the sources are unchanged since the last build, reuse)
    the host-sanitizer library; returns its path."""
    out = os.path.dirname(HOSTSAN_LIB)
    os.makedirs(out, exist_ok=True)
    stamp_file = HOSTSAN_LIB + ".stamp"
    stamp = _hostsan_stamp()
    if not force and os.path.exists(HOSTSAN_LIB) and os.path.exists(stamp_file):
        with open(stamp_file) as fh:
            if fh.read() == stamp:
                return HOSTSAN_LIB

    def one(src):
        obj = os.path.join(out, os.path.basename(src)[:-4] + ".o")
        r = subprocess.run([hipcc()] + HOSTSAN_FLAGS + ["-c", src, "-o", obj],
                           capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"host sanitizer build failed on {src}:\n{r.stderr}")
        return obj

    srcs = sources()
    workers = min(len(srcs), int(os.environ.get("MAX_JOBS", "8")), 16)
    with concurrent.futures.ThreadPoolExecutor(max_workers=max(workers, 1)) as ex:
        objs = list(ex.map(one, srcs))
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-shared-libsan", "-o", HOSTSAN_LIB] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"host sanitizer link failed:\n{r.stdout}\n{r.stderr}")
    with open(stamp_file, "w") as fh:
        fh.write(stamp)
    if verbose:
        print(f"built {HOSTSAN_LIB}")
    return HOSTSAN_LIB


if __name__ == "__main__":
    if "--hostsan" in sys.argv:
        build_hostsan(verbose=True, force=True)
    else:
        build()
