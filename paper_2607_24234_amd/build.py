"""Build libqs.so (the HIP library behind include/qs.h) for gfx950 with hipcc, in-tree."""
from __future__ import annotations

import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libqs.so")
ARCH = os.environ.get("QS_OFFLOAD_ARCH", "gfx950")

# Packed FP32 instructions stay disabled on every HIP source of this library.
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", os.path.join(ROOT, "include")]


def sources():
    return sorted(glob.glob(os.path.join(PKG, "csrc", "*.hip")))


# Host-side sanitizers for a CPU-only test build (the device code is compiled as usual): each
# -fsanitize applies to the host compilation only.
HOST_SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
                 "-Xarch_host", "-g"]


def build(verbose: bool = False, out: str = LIB, defines=(), objdir=None, sanitize: bool = False) -> str:
    """Compile every HIP source into libqs.so (always rebuilds).  sanitize: instrument the
    host code with AddressSanitizer and UndefinedBehaviorSanitizer (a CPU test build: the
    process that loads it needs clang's ASan runtime first, LD_PRELOAD)."""
    objdir = objdir or os.path.join(PKG, "_build" if not sanitize else "_build_san")
    os.makedirs(objdir, exist_ok=True)
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    extra = HOST_SANITIZE if sanitize else []
    cmds, objs = [], []
    for src in sources():
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        cmds.append([hipcc, *HIP_FLAGS, *extra, *["-D" + d for d in defines], "-c", src, "-o", obj])
        objs.append(obj)
    if verbose:
        for cmd in cmds:
            print(" ".join(cmd), flush=True)
    # one compiler process per source, at most as many as the machine's share of cores
    jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with ThreadPoolExecutor(jobs) as pool:
        for f in [pool.submit(subprocess.check_call, cmd) for cmd in cmds]:
            f.result()
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [hipcc, "--offload-arch=" + ARCH, "-shared", "-fPIC", *extra, "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
