"""Host-side checks of bench.py's command-line contract (no GPU needed)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args, env=None):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, env=env)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = _run("--gpus", "2", "--steps", "5", "--warmup", "1")
    assert r.returncode == 2
    assert "one MI355X" in r.stderr
    env = dict(os.environ, WORLD_SIZE="4")
    r = _run("--gpus", "1", env=env)
    assert r.returncode == 2


def test_help_lists_the_workloads_and_the_legs():
    r = _run("--help")
    assert r.returncode == 0
    for flag in ("--workload", "--steps", "--warmup", "--no-theta4", "--no-pipelined", "--copy-probe"):
        assert flag in r.stdout, flag
