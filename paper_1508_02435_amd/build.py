"""Build libpic.so (the HIP kernels and the C ABI) for gfx950 with hipcc.

Run as ``python -m paper_1508_02435_amd.build``.  Every source is compiled to
an object file in parallel (the kernel sources take most of the time), then
the objects are linked.  The library is built in place, next to this file,
so that it travels with the source tree; objects go to ``_build/``.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libpic.so")
SOURCES = ["pic_tree.hip", "pic_kernels.hip", "pic_rebin.hip", "pic_rank.hip", "pic_step.hip", "pic_f32.hip",
           "pic_stats.hip", "pic_move.hip", "pic_capi.hip", "pic_profile.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC",
    # the FP64 path promises the exact IEEE operation sequence: no contraction
    "-ffp-contract=off",
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


# host code only: AddressSanitizer and UndefinedBehaviorSanitizer (every
# option behind -Xarch_host, so the device code is built as always)
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
            "-Xarch_host", "-g"]
SAN_LINK = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-shared-libsan"]


def _compile(src: str, verbose: bool, sanitize: bool = False) -> str:
    odir = OBJ + "_san" if sanitize else OBJ
    obj = os.path.join(odir, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, *(SAN_HOST if sanitize else []), "-I", os.path.join(HERE, "..", "include"), "-c", "-o",
           obj, os.path.join(CSRC, src)]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed on {src}")
    return obj


def build(verbose: bool = False, jobs: int = 0, sanitize: bool = False) -> str:
    """Build libpic.so; with ``sanitize`` build libpic_san.so instead, whose
    host code runs under AddressSanitizer and UndefinedBehaviorSanitizer
    (load it with PIC_LIBPIC in a process that preloads clang's ASan
    runtime)."""
    os.makedirs(OBJ + "_san" if sanitize else OBJ, exist_ok=True)
    out = os.path.join(HERE, "libpic_san.so") if sanitize else LIB
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 4, 16)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, sanitize), SOURCES))
    tmp = out + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *(SAN_LINK if sanitize else []), "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed linking libpic.so")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True, sanitize="--sanitize" in sys.argv[1:]))
