"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer:
the table builders, and the host side of the C ABI (second test below).

tests/sanitize/host_tables.cpp calls the chart-T radial and polar table
builder, the chart-H per-point table builder and the double-double
(binary128) table builder on about a thousand configurations: grids from
7 x 2 to 4097 x 16, a = 0 .. M, s = -2 .. 2, |m| up to 8, radial ranges
reaching deep towards the horizon.  Built with g++ (host code only; no GPU
code is instrumented), any out-of-bounds access, use after free, leak,
overflow or other undefined behaviour aborts the run; every table built
must also be finite."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2010_04760_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_table_builders_clean_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "host_tables")
    cmd = ["g++", "-std=gnu++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
           os.path.join(ROOT, "tests", "sanitize", "host_tables.cpp"), os.path.join(CSRC, "teuk_background.cpp"),
           os.path.join(CSRC, "teuk_background_dd.cpp"), "-lquadmath", "-o", exe]
    b = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert b.returncode == 0, b.stderr[-3000:]
    # the ASan runtime is linked into the executable; a library the environment preloads
    # ahead of it is tolerated rather than treated as an error
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "failures 0" in r.stdout, r.stdout


def _load_build():
    import importlib.util
    spec = importlib.util.spec_from_file_location("_teuk_build", os.path.join(ROOT, "paper_2010_04760_amd", "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.skipif(shutil.which("hipcc") is None or shutil.which("g++") is None, reason="hipcc or g++ missing")
def test_abi_host_code_clean_under_asan_and_ubsan(tmp_path):
    """tests/sanitize/host_abi.cpp drives the host side of the C ABI:
    validation with every field pushed out of range, footprints, the host
    evaluation of the coefficients (chart T, chart H, double-double) and
    teuk_create / teuk_destroy (which fail cleanly where no GPU answers).
    teuk_api.hip and teuk_tune.hip are compiled with the sanitizers on their
    host pass only; the kernels come unchanged from the library's own build."""
    clang = "/opt/rocm/llvm/bin/clang++"
    if not os.path.exists(clang):
        pytest.skip("ROCm clang++ missing")
    bdir = os.path.join(ROOT, "_build")
    kernels = [os.path.join(bdir, f) for f in ("teuk_kernels.hip.o", "teuk_kernels_dd.hip.o", "teuk_kernels_cmp.hip.o")]
    srcs = [os.path.join(CSRC, f) for f in os.listdir(CSRC)]
    if not all(os.path.exists(k) for k in kernels) or \
            max(os.path.getmtime(s) for s in srcs) > min(os.path.getmtime(k) for k in kernels):
        _load_build().build()
    inc = ["-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer"]
    objs = []
    jobs = []
    for f in ("teuk_api.hip", "teuk_tune.hip"):
        o = str(tmp_path / (f + ".o"))
        jobs.append(["hipcc", "--offload-arch=gfx950", "-std=c++17", "-O1", "-g", "-fPIC", "-Xclang", "-target-feature",
                     "-Xclang", "-packed-fp32-ops", *san, *inc, "-c", os.path.join(CSRC, f), "-o", o])
        objs.append(o)
    o = str(tmp_path / "teuk_background.o")
    jobs.append([clang, "-std=gnu++17", "-O1", "-g", "-fPIC", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                 *inc, "-c", os.path.join(CSRC, "teuk_background.cpp"), "-o", o])
    objs.append(o)
    o = str(tmp_path / "teuk_background_dd.o")      # binary128 code: g++ and libquadmath, not instrumented here
    jobs.append(["g++", "-std=gnu++17", "-O1", "-g", "-fPIC", *inc, "-c", os.path.join(CSRC, "teuk_background_dd.cpp"),
                 "-o", o])
    objs.append(o)
    o = str(tmp_path / "host_abi.o")
    jobs.append([clang, "-std=gnu++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                 "-I" + os.path.join(ROOT, "include"), "-c", os.path.join(ROOT, "tests", "sanitize", "host_abi.cpp"),
                 "-o", o])
    objs.append(o)
    procs = [subprocess.Popen(j, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True) for j in jobs]
    for j, p in zip(jobs, procs):
        _, err = p.communicate(timeout=600)
        assert p.returncode == 0, (j[-1], err[-3000:])
    exe = str(tmp_path / "host_abi")
    link = [clang, "-fsanitize=address,undefined", *objs, *kernels, "-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib",
            "-lamdhip64", "-lquadmath", "-o", exe]
    b = subprocess.run(link, capture_output=True, text=True, timeout=600)
    assert b.returncode == 0, b.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "failures 0" in r.stdout, r.stdout
