"""Graph mode (teuk_set_graph / teuk_group_set_graph) against stepping launch
by launch.

A solver in graph mode replays a captured graph of chunk steps and runs the
remainder launch by launch; its state, waveform ring, horizon ring, times and
counters must equal those of an identical solver stepped without graphs, bit
for bit, after every call.  The call sequences replay the graph several times
with synchronising extractions between calls, leave eager remainders that
shift the sampling phase (which forces a recapture), and wrap the waveform
ring.
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
    return T.make_config(s=wl.s, m=wl.m, a=wl.a, nr=wl.nr, ntheta=wl.nth, x_min=wl.x_min, x_max=wl.x_max,
                         chart=wl.chart, S=wl.S, **kw)


def _pair(wl, **kw):
    """Two identical solvers (same explicit dt), the first in graph mode."""
    with T.Solver(_cfg(wl, **{k: v for k, v in kw.items() if k not in ("extract_every", "max_samples", "x_extract")})) as p:
        dt = p.info().dt
    cfg = _cfg(wl, dt=dt, **kw)
    u0 = W.gaussian_pulse(wl)
    a, b = T.Solver(cfg), T.Solver(cfg)
    a.set_initial(u0)
    b.set_initial(u0)
    return a, b


def _same(a, b, chart_h=False):
    ia, ib = a.info(), b.info()
    assert (ia.steps, ia.samples) == (ib.steps, ib.samples)
    np.testing.assert_array_equal(a.state(), b.state())
    ta, wa = a.waveform()
    tb, wb = b.waveform()
    np.testing.assert_array_equal(ta, tb)
    np.testing.assert_array_equal(wa, wb)
    if chart_h:
        for x, y in zip(a.horizon(), b.horizon()):
            np.testing.assert_array_equal(x, y)


CALLS = [30, 12, 10, 7, 20, 3, 40]


@pytest.mark.parametrize("integrator,chunk,every", [("rk3", 10, 5), ("rk3_blocked", 4, 2), ("rk104", 6, 3)])
def test_single_solve_graph_equals_eager(integrator, chunk, every):
    wl = W.C1.with_(nr=300, nth=24)
    a, b = _pair(wl, integrator=integrator, extract_every=every, max_samples=7, x_extract=10.0)
    a.set_graph(chunk)
    for n in CALLS:
        say(f"{integrator} chunk {chunk} every {every}: step {n}")
        a.step(n)
        b.step(n)
        _same(a, b)
    a.close()
    b.close()


@pytest.mark.parametrize("every", [0, 3])
def test_blocked_graph_after_odd_eager_steps(every):
    """The blocked step trades its two state buffers every step, and a graph
    holds the buffers of its capture.  With no waveform, or an odd sampling
    interval, an odd number of eager steps between replays leaves the
    sampling phase unchanged but the buffers traded: the next replay must
    recapture (it would otherwise start from the stale buffer)."""
    wl = W.C1.with_(nr=300, nth=24)
    kw = dict(extract_every=every, max_samples=9 if every else 0, x_extract=10.0)
    a, b = _pair(wl, integrator="rk3_blocked", **kw)
    a.set_graph(6)
    for n in (3, 6, 9, 12, 5, 7, 6):
        say(f"blocked every {every}: step {n}")
        a.step(n)
        b.step(n)
        _same(a, b)
    a.close()
    b.close()


def test_chart_h_graph_equals_eager():
    wl = W.C3H.with_(nr=240, nth=16)
    a, b = _pair(wl, extract_every=5, max_samples=9, x_extract=19.0)
    a.set_graph(10)
    for n in CALLS:
        say(f"chart H: step {n}")
        a.step(n)
        b.step(n)
        _same(a, b, chart_h=True)
    a.close()
    b.close()


def test_graph_mode_off_again_and_mixed_weights():
    wl = W.C2.with_(nr=400, nth=32, x_min=-100.0, x_max=200.0)
    a, b = _pair(wl, weight_prec="fp32", extract_every=10, max_samples=50, x_extract=30.0)
    a.set_graph(20)
    a.step(40)
    b.step(40)
    _same(a, b)
    a.set_graph(0)
    a.step(15)
    b.step(15)
    _same(a, b)
    a.set_graph(10)
    a.step(25)
    b.step(25)
    _same(a, b)
    a.close()
    b.close()


def test_group_graph_equals_eager():
    specs = [W.C2.with_(nr=500, nth=40, x_min=-100.0, x_max=200.0, seed=31),
             W.C1.with_(nr=260, nth=20, seed=32),
             W.C2.with_(nr=320, nth=64, s=0, m=1, a=0.7, x_min=-80.0, x_max=150.0, seed=33)]
    wps = ["fp64", "fp32", "fp64"]
    ga, gb = T.Group(4), T.Group(4)
    A, B = [], []
    for wl, wp in zip(specs, wps):
        a, b = _pair(wl, weight_prec=wp, extract_every=5, max_samples=6, x_extract=20.0)
        ga.add(a)
        gb.add(b)
        A.append(a)
        B.append(b)
    ga.set_graph(10)
    for n in CALLS:
        say(f"group: step {n}")
        ga.step(n)
        gb.step(n)
        for a, b in zip(A, B):
            _same(a, b)
    # membership change drops the graphs; stepping recaptures
    ga.remove(A[1])
    gb.remove(B[1])
    ga.step(20)
    gb.step(20)
    for a, b in zip(A, B):
        _same(a, b)
    ga.close()
    gb.close()
    for x in A + B:
        x.close()


def test_graph_errors():
    wl = W.C1.with_(nr=120, nth=12)
    cfg = _cfg(wl, extract_every=4, max_samples=4, x_extract=10.0)
    with T.Solver(cfg) as sv:
        sv.set_initial(W.gaussian_pulse(wl))
        with pytest.raises(T.TeukError) as ei:
            sv.set_graph(6)                                  # not a multiple of extract_every
        assert ei.value.status == T.TEUK_ERR_INVALID_ARG
        with pytest.raises(T.TeukError) as ei:
            sv.set_graph(5000)
        assert ei.value.status == T.TEUK_ERR_INVALID_ARG
        sv.set_graph(8)
        sv.step(16)
    with T.Solver(_cfg(wl, integrator="rk3_blocked")) as sv:
        with pytest.raises(T.TeukError) as ei:
            sv.set_graph(3)
        assert ei.value.status == T.TEUK_ERR_INVALID_ARG
    with T.Solver(_cfg(wl, state="dd", weight_prec="fp64")) as sv:
        with pytest.raises(T.TeukError) as ei:
            sv.set_graph(4)
        assert ei.value.status == T.TEUK_ERR_UNSUPPORTED
    # a group member whose cadence does not divide the chunk is refused: at
    # set_graph when it is already a member, at step time when it joins later
    g = T.Group(2)
    sv = T.Solver(_cfg(wl, extract_every=3, max_samples=4, x_extract=10.0))
    sv.set_initial(W.gaussian_pulse(wl))
    g.add(sv)
    with pytest.raises(T.TeukError) as ei:
        g.set_graph(8)
    assert ei.value.status == T.TEUK_ERR_INVALID_ARG
    g.remove(sv)
    g.set_graph(8)
    g.add(sv)
    with pytest.raises(T.TeukError) as ei:
        g.step(8)
    assert ei.value.status == T.TEUK_ERR_INVALID_ARG
    g.close()
    sv.close()
    torch.cuda.synchronize()
