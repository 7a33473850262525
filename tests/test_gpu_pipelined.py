"""Pipelined steps (TEUK_RK_SSP33_PIPELINED) against the three-launch step.

The pipelined integrator runs the tiles of the three stage launches inside one
cooperative launch, each tile waiting for its neighbours' previous stage
through device-memory counters.  It runs the same per-point arithmetic, so its
state and waveform must equal those of TEUK_RK_SSP33 bit for bit; any
dependency or memory-visibility fault would show up as a mismatch (stale
values of an earlier stage or step) or as the timed-out-wait error.  Cases
cover ragged and minimal grids, the waveform cadence splitting launches, the
C2 grid at full size, repeated runs, and the error paths.
"""
import numpy as np
import pytest
import torch

import paper_2010_04760_amd as T
import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def _cfg(wl, **kw):
    return T.make_config(s=wl.s, m=wl.m, a=wl.a, nr=wl.nr, ntheta=wl.nth, x_min=wl.x_min, x_max=wl.x_max, **kw)


def _run(wl, integrator, calls, u0=None, **kw):
    with T.Solver(_cfg(wl, integrator="rk3", **{k: v for k, v in kw.items()
                                                   if k not in ("extract_every", "max_samples", "x_extract")})) as p:
        dt = p.info().dt
    with T.Solver(_cfg(wl, integrator=integrator, dt=dt, **kw)) as sv:
        sv.set_initial(W.gaussian_pulse(wl) if u0 is None else u0)
        for n in calls:
            sv.step(n)
        st = sv.state()
        wave = sv.waveform()[1] if kw.get("extract_every", 0) else None
        return st, wave, sv.info()


CASES = [
    ("C1", W.C1, {}),
    ("ragged 130x7", W.C1.with_(nr=130, nth=7, seed=61), {}),
    ("minimal 7x2", W.C1.with_(nr=7, nth=2, seed=62), {}),
    ("extremal 2000x40 s=-2 m=2", W.C2.with_(nr=2000, nth=40, a=1.0, x_min=-150.0, x_max=250.0, seed=63), {}),
    ("fp32 weights 1000x64", W.C2.with_(nr=1000, nth=64, x_min=-100.0, x_max=200.0, seed=64), {"weight_prec": "fp32"}),
    ("fp16 weights 640x33 m=1", W.C2.with_(nr=640, nth=33, m=1, x_min=-100.0, x_max=200.0, seed=65), {"weight_prec": "fp16"}),
    ("bf16 weights 900x18 m=3", W.C2.with_(nr=900, nth=18, m=3, x_min=-100.0, x_max=200.0, seed=66), {"weight_prec": "bf16"}),
]


@pytest.mark.parametrize("name,wl,kw", CASES, ids=[c[0] for c in CASES])
def test_pipelined_equals_three_launch(name, wl, kw):
    calls = [7, 13, 1, 25]
    say(f"pipelined vs rk3: {name}, calls {calls}")
    a, _, ia = _run(wl, "rk3_pipelined", calls, **kw)
    b, _, ib = _run(wl, "rk3", calls, **kw)
    assert ia.steps == ib.steps == sum(calls)
    assert np.all(np.isfinite(a))
    np.testing.assert_array_equal(a, b)


def test_pipelined_waveform_cadence_splits_launches():
    wl = W.C2.with_(nr=1500, nth=48, x_min=-100.0, x_max=200.0, seed=66)
    kw = dict(extract_every=7, max_samples=9, x_extract=20.0)
    calls = [10, 4, 30]
    a, wa, ia = _run(wl, "rk3_pipelined", calls, **kw)
    b, wb, ib = _run(wl, "rk3", calls, **kw)
    assert ia.samples == ib.samples
    np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(wa, wb)


def test_pipelined_full_c2_grid_repeated():
    wl = W.C2
    b, _, _ = _run(wl, "rk3", [30])
    for trial in range(3):
        say(f"pipelined C2 8192x256, 30 steps, trial {trial}")
        a, _, info = _run(wl, "rk3_pipelined", [30])
        np.testing.assert_array_equal(a, b)
    say(f"pipelined C2: {info.workgroups} workgroups")


def test_pipelined_not_offered():
    wl = W.C1.with_(nr=100, nth=10)
    with T.Solver(_cfg(wl, integrator="rk3_pipelined")) as sv:
        with pytest.raises(T.TeukError) as ei:
            sv.set_graph(10)
        assert ei.value.status == T.TEUK_ERR_UNSUPPORTED
    for kw in (dict(state="dd", weight_prec="fp64"), dict(scheme="weno3")):
        with pytest.raises(T.TeukError) as ei:
            T.Solver(_cfg(wl, integrator="rk3_pipelined", **kw))
        assert ei.value.status == T.TEUK_ERR_UNSUPPORTED
    wh = W.C3H.with_(nr=200, nth=8)
    with pytest.raises(T.TeukError) as ei:
        T.Solver(T.make_config(s=wh.s, m=wh.m, a=wh.a, nr=wh.nr, ntheta=wh.nth, x_min=wh.x_min, x_max=wh.x_max,
                               chart="H", integrator="rk3_pipelined"))
    assert ei.value.status == T.TEUK_ERR_UNSUPPORTED
    torch.cuda.synchronize()
