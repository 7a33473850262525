"""Build libteuk.so (HIP, gfx950) in the package directory with hipcc.

This file imports nothing from the package, so it can be loaded by path (and
run as a script) before the library exists.  Each translation unit is compiled
to an object of its own, in parallel, and the objects are then linked; no unit
launches a kernel defined in another, so no relocatable device code is needed.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libteuk.so")
SOURCES = ["teuk_api.hip", "teuk_tune.hip", "teuk_kernels.hip", "teuk_kernels_dd.hip", "teuk_kernels_cmp.hip", "teuk_background.cpp"]
# host-only sources that need the GNU C++ compiler (binary128 via libquadmath)
GXX_SOURCES = ["teuk_background_dd.cpp"]
GXX_FLAGS = ["-O2", "-std=gnu++17", "-fPIC", "-Wall", "-fno-fast-math"]
BUILD_DIR = os.path.join(ROOT, "_build")

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # code object v5 is understood by both the ROCm 7.2 toolchain and the
    # ROCm 7.0 runtime that ships inside the PyTorch wheel
    "-mcode-object-version=5",
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-function",
]


def _run(cmd: list[str], what: str, verbose: bool) -> None:
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    # the host pass warns that it does not know the device-only feature above
    msgs = [ln for ln in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in ln]
    if r.returncode != 0:
        sys.stderr.write("\n".join(msgs) + "\n")
        raise RuntimeError(f"{what} failed (exit {r.returncode})")
    if verbose and msgs:
        print("\n".join(msgs), flush=True)


def build(verbose: bool = False, extra_flags: list[str] | None = None) -> str:
    """Compile every source and link libteuk.so; returns its path.  Raises
    RuntimeError (with the compiler's messages on stderr) if any step fails."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include")]
    jobs = []
    for s in GXX_SOURCES:
        obj = os.path.join(BUILD_DIR, os.path.splitext(s)[0] + ".o")
        jobs.append((["g++", *GXX_FLAGS, *inc, "-c", os.path.join(CSRC, s), "-o", obj], f"g++ {s}", obj))
    for s in SOURCES:
        obj = os.path.join(BUILD_DIR, os.path.splitext(s)[0] + ".hip.o")
        jobs.append((["hipcc", *HIPCC_FLAGS, *(extra_flags or []), *inc, "-c", os.path.join(CSRC, s), "-o", obj],
                     f"hipcc {s}", obj))
    with ThreadPoolExecutor(max_workers=min(len(jobs), 8)) as ex:
        for f in [ex.submit(_run, cmd, what, verbose) for cmd, what, _ in jobs]:
            f.result()
    tmp = LIB + ".tmp"
    objs = [o for _, _, o in jobs]
    _run(["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-lquadmath", "-o", tmp],
         "linking libteuk.so", verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
