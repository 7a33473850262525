"""The library's host-side table builders under AddressSanitizer and
UndefinedBehaviorSanitizer.

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
