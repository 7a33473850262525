"""Launch-shape autotuner (teuk_tune, teuk_group_tune).

The tuner picks among launch shapes whose tiles run the same per-point
arithmetic, so a solver on the tuned shape must equal one on the default
shape bit for bit; a tuned budget must reach later solvers of the same launch
class (and only those) and be forgotten on request; the group tuner must not
advance or perturb the members it tunes on.
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


def _run(cfg, u0, n):
    with T.Solver(cfg) as sv:
        sv.set_initial(u0)
        sv.step(n)
        return sv.state(), sv.info().workgroups


@pytest.mark.parametrize("integrator,strip", [("rk3", 63), ("rk3_blocked", 114)])
def test_tuned_shape_equals_default_and_is_remembered(integrator, strip):
    T.teuk_tune_forget()
    wl = W.C2.with_(nr=2048, nth=96, x_min=-100.0, x_max=200.0, seed=41)
    with T.Solver(_cfg(wl, integrator=integrator)) as p:
        dt = p.info().dt
    cfg = _cfg(wl, integrator=integrator, dt=dt)
    u0 = W.gaussian_pulse(wl)
    ref, wg_default = _run(cfg, u0, 30)
    info = T.teuk_tune(cfg, 10)
    say(f"{integrator}: {info.candidates} candidates, best budget {info.workgroups} (segs {info.segs}) "
        f"{info.us_per_step:.1f} us/step, default {info.default_workgroups} (segs {info.default_segs}) "
        f"{info.us_per_step_default:.1f} us/step")
    assert info.candidates >= 3 and info.steps == 10
    assert info.us_per_step > 0 and info.us_per_step <= info.us_per_step_default
    nstrips = (wl.nr + strip - 1) // strip
    got, wg = _run(cfg, u0, 30)
    assert wg == nstrips * info.segs                       # the tuned budget is in use
    np.testing.assert_array_equal(got, ref)
    # another launch class is not affected
    other = _cfg(wl.with_(nth=64), integrator=integrator, dt=dt)
    _, wg_other = _run(other, W.gaussian_pulse(wl.with_(nth=64)), 1)
    T.teuk_tune_forget()
    _, wg_other_default = _run(other, W.gaussian_pulse(wl.with_(nth=64)), 1)
    assert wg_other == wg_other_default
    _, wg_after = _run(cfg, u0, 1)
    assert wg_after == wg_default


def test_tune_rejects_double_double():
    wl = W.C1.with_(nr=120, nth=12)
    with pytest.raises(T.TeukError) as ei:
        T.teuk_tune(_cfg(wl, state="dd", weight_prec="fp64"), 2)
    assert ei.value.status == T.TEUK_ERR_UNSUPPORTED


def test_group_tune_leaves_members_and_results_unchanged():
    specs = [W.C2.with_(nr=700, nth=48, x_min=-100.0, x_max=200.0, seed=51),
             W.C2.with_(nr=1200, nth=80, s=0, m=1, a=0.6, x_min=-100.0, x_max=200.0, seed=52),
             W.C1.with_(nr=400, nth=40, seed=53)]

    def members():
        out = []
        for wl in specs:
            sv = T.Solver(_cfg(wl, weight_prec="fp32", extract_every=5, max_samples=20, x_extract=20.0))
            sv.set_initial(W.gaussian_pulse(wl))
            out.append(sv)
        return out

    A, B = members(), members()
    ga, gb = T.Group(4), T.Group(4)
    for a, b in zip(A, B):
        ga.add(a)
        gb.add(b)
    ga.step(7)
    gb.step(7)
    before = [a.state() for a in A]
    info = ga.tune(3)
    say(f"group tune: {info.candidates} shapes, best rows {info.rows_per_tile} block {info.block_mib} MiB "
        f"{info.us_per_step:.1f} us/step; default rows {info.default_rows_per_tile} block "
        f"{info.default_block_mib} MiB {info.us_per_step_default:.1f} us/step")
    assert info.candidates >= 10 and info.us_per_step <= info.us_per_step_default
    for a, s in zip(A, before):
        assert a.info().steps == 7
        np.testing.assert_array_equal(a.state(), s)
    ga.step(20)
    gb.step(20)
    for a, b in zip(A, B):
        np.testing.assert_array_equal(a.state(), b.state())
        ta, wa = a.waveform()
        tb, wb = b.waveform()
        np.testing.assert_array_equal(wa, wb)
    ga.close()
    gb.close()
    for x in A + B:
        x.close()
    torch.cuda.synchronize()
