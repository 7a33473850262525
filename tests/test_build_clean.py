"""The library builds from a clean tree (no built files), through the build
entry point and through a bare package import.

The tree is the set of files git would commit (tracked plus untracked files
that .gitignore does not list), copied to a temporary directory, so built
libraries and build folders of this working copy are left behind.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _committed_files():
    r = subprocess.run(["git", "ls-files", "-z", "--cached", "--others", "--exclude-standard"],
                       cwd=ROOT, capture_output=True)
    if r.returncode != 0:
        pytest.skip("not a git checkout")
    return [f for f in r.stdout.decode().split("\0") if f and os.path.isfile(os.path.join(ROOT, f))]


def _copy_tree(dst):
    files = _committed_files()
    for f in files:
        assert not f.endswith(".so"), f"a built library is committed: {f}"
        os.makedirs(os.path.join(dst, os.path.dirname(f)), exist_ok=True)
        shutil.copy2(os.path.join(ROOT, f), os.path.join(dst, f))


def _py(cwd, code, timeout=600):
    env = dict(os.environ)
    env.pop("PYTHONPATH", None)
    r = subprocess.run([sys.executable, "-c", code], cwd=cwd, capture_output=True, text=True,
                       timeout=timeout, env=env)
    assert r.returncode == 0, f"exit {r.returncode}\n--- stdout\n{r.stdout[-3000:]}\n--- stderr\n{r.stderr[-3000:]}"
    return r.stdout


@pytest.mark.skipif(shutil.which("hipcc") is None or shutil.which("git") is None, reason="needs hipcc and git")
def test_build_entry_and_lazy_import_from_clean_tree(tmp_path):
    tree = str(tmp_path / "repo")
    _copy_tree(tree)
    lib = os.path.join(tree, "paper_2010_04760_amd", "libteuk.so")
    assert not os.path.exists(lib)

    # the build entry point on a tree with nothing built
    _py(tree, "import __graft_entry__ as g; g.build()")
    for f in ("paper_2010_04760_amd/libteuk.so", "oracle/_liboracle.so", "oracle/_liboracle_q.so"):
        assert os.path.isfile(os.path.join(tree, f)), f
    out = _py(tree, "import paper_2010_04760_amd as T, ctypes\n"
                    "L = ctypes.CDLL(T.LIB_PATH)\n"
                    "print(T.LIB_PATH); print(all(hasattr(L, n) for n in T.EXPORTED))")
    assert out.split()[0] == lib and out.split()[1] == "True"

    # a bare import of the package builds the library when it is missing
    os.remove(lib)
    out = _py(tree, "import paper_2010_04760_amd as T; print(T.LIB_PATH)")
    assert out.strip().splitlines()[-1] == lib and os.path.isfile(lib)
