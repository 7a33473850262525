"""Build libteuk.so (HIP, gfx950) in the package directory with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libteuk.so")
SOURCES = ["teuk_api.hip", "teuk_kernels.hip", "teuk_kernels_dd.hip", "teuk_kernels_cmp.hip", "teuk_background.cpp"]
# host-only sources that need the GNU C++ compiler (binary128 via libquadmath)
GXX_SOURCES = ["teuk_background_dd.cpp"]
GXX_FLAGS = ["-O2", "-std=gnu++17", "-fPIC", "-Wall", "-fno-fast-math"]
BUILD_DIR = os.path.join(ROOT, "_build")

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # code object v5 is understood by both the ROCm 7.2 toolchain and the
    # ROCm 7.0 runtime that ships inside the PyTorch wheel
    "-mcode-object-version=5",
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-function",
]


def build(verbose: bool = False, extra_flags: list[str] | None = None) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    os.makedirs(BUILD_DIR, exist_ok=True)
    objs = []
    for s in GXX_SOURCES:
        obj = os.path.join(BUILD_DIR, os.path.splitext(s)[0] + ".o")
        gcmd = ["g++", *GXX_FLAGS, "-I", os.path.join(ROOT, "include"), "-c", os.path.join(CSRC, s), "-o", obj]
        if verbose:
            print(" ".join(gcmd), flush=True)
        r = subprocess.run(gcmd, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError(f"g++ failed building {s}")
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = ["hipcc", *HIPCC_FLAGS, *(extra_flags or []), "-I", os.path.join(ROOT, "include"), *srcs, *["-Wl," + o for o in objs],
           "-lquadmath", "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    # the host pass warns that it does not know the device-only feature above
    msgs = [ln for ln in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in ln]
    if r.returncode != 0:
        sys.stderr.write("\n".join(msgs) + "\n")
        raise RuntimeError("hipcc failed building libteuk.so")
    if verbose and msgs:
        print("\n".join(msgs))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
