"""The explicitly waited loads of the stage kernels are safe in the built code.

The tortoise-chart stage kernel issues the u^n loads of a row from inline
assembly and waits for them later with an explicit `s_waitcnt` that takes the
four values as operands.  The compiler takes an asm output as ready at once, so
if it copied, spilled or reused one of those registers before the wait, the
kernel would read a value still in flight.  This test compiles the kernels to
gfx950 assembly with the library's own flags and checks, on the control-flow
graph of every kernel, that on every path from such a load to its wait no
instruction mentions the load's destination registers.  The loads and waits
mark themselves with the comments "async-load" and "async-wait <operands>".
"""
import importlib.util
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2010_04760_amd", "csrc", "teuk_kernels.hip")

_REG = re.compile(r"\bv\[(\d+):(\d+)\]|\bv(\d+)\b")
_LABEL = re.compile(r"^(\.?[A-Za-z_][\w.$]*):")


def _regs(text):
    out = set()
    for a, b, c in _REG.findall(text):
        if c:
            out.add(int(c))
        else:
            out.update(range(int(a), int(b) + 1))
    return out


def _code(line):
    return line.split(";", 1)[0].strip()


def _functions(asm_lines):
    """Yield (name, [lines]) for every kernel body in the assembly."""
    name, body = None, []
    for ln in asm_lines:
        m = _LABEL.match(ln)
        if m and not m.group(1).startswith("."):
            if name is not None:
                yield name, body
            name, body = m.group(1), []
            continue
        if name is not None:
            body.append(ln.rstrip("\n"))
            if ln.strip().startswith(".Lfunc_end"):
                yield name, body
                name, body = None, []
    if name is not None:
        yield name, body


def _cfg(body):
    """Instruction list, label -> index, and successors of each index."""
    ins, labels = [], {}
    for ln in body:
        s = ln.strip()
        m = _LABEL.match(s)
        if m:
            labels[m.group(1)] = len(ins)
            continue
        if not s or s.startswith((".", ";")):
            continue
        ins.append(s)
    succ = []
    for i, s in enumerate(ins):
        op = _code(s).split()[0] if _code(s) else ""
        nxt = [i + 1] if i + 1 < len(ins) else []
        if op == "s_branch":
            nxt = [labels[_code(s).split()[1]]]
        elif op.startswith("s_cbranch"):
            nxt = nxt + [labels[_code(s).split()[1]]]
        elif op in ("s_endpgm", "s_setpc_b64"):
            nxt = []
        succ.append(nxt)
    return ins, succ


def _check_function(name, body):
    ins, succ = _cfg(body)
    loads = [i for i, s in enumerate(ins) if "async-load" in s]
    waits = [i for i, s in enumerate(ins) if "async-wait" in s]
    problems = []
    for li in loads:
        dest = _regs(_code(ins[li]).split(",")[0])
        assert len(dest) == 2, ins[li]
        # walk every path from the load; a path ends at a wait naming these registers
        seen, stack, reached = set(), list(succ[li]), False
        while stack:
            i = stack.pop()
            if i in seen:
                continue
            seen.add(i)
            s = ins[i]
            if "async-wait" in s and dest <= _regs(s.split("async-wait", 1)[1]):
                reached = True
                continue
            if dest & _regs(_code(s)):
                problems.append(f"{name}: {ins[li]!r} -> {s!r} before its wait")
                continue
            stack.extend(succ[i])
        if not reached:
            problems.append(f"{name}: {ins[li]!r} reaches no wait naming its registers")
    return len(loads), len(waits), problems


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="needs hipcc")
def test_async_load_registers_untouched_until_their_wait(tmp_path):
    spec = importlib.util.spec_from_file_location("_teuk_build", os.path.join(ROOT, "paper_2010_04760_amd", "build.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    flags = [f for f in b.HIPCC_FLAGS if f not in ("-fPIC",)]
    out = tmp_path / "k.s"
    r = subprocess.run(["hipcc", *flags, "-I", os.path.join(ROOT, "include"), "-S", "--offload-device-only", SRC,
                        "-o", str(out)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    lines = out.read_text().splitlines()
    total_loads, total_waits, problems = 0, 0, []
    for name, body in _functions(lines):
        nl, nw, p = _check_function(name, body)
        total_loads += nl
        total_waits += nw
        problems += p
    assert total_loads > 0 and total_waits > 0, "no explicitly waited loads found in the assembly"
    assert not problems, "\n".join(problems[:20])


def test_checker_flags_a_copy_before_the_wait():
    """The checker itself: a copy of an in-flight register is reported, a use
    after the wait and a branch around unrelated code are not."""
    good = ["\tglobal_load_dwordx2 v[4:5], v1, s[0:1] ; async-load",
            "\ts_cbranch_execz .LBB0_2",
            "\tv_mov_b32_e32 v7, v8",
            ".LBB0_2:",
            "\ts_waitcnt vmcnt(0) ; async-wait v[4:5] v[6:7] v[8:9] v[10:11]",
            "\tv_mov_b32_e32 v12, v4",
            "\ts_endpgm"]
    assert _check_function("k", good)[2] == []
    bad = list(good)
    bad[2] = "\tv_mov_b32_e32 v7, v5"
    assert len(_check_function("k", bad)[2]) == 1
