"""Allocation-free stepping (teuk_step_noalloc) against teuk_step.

The entry point advances a caller-held device state with its stage buffers
and coefficient tables in the library's fixed device array.  It runs the same
stage kernels with the same launch shapes as a solver created with the same
configuration, so the two results must agree bit for bit.  Two calls in a row
on different grids (the second smaller) check that the array's previous
contents do not leak into the next call, and a third call repeats the first
grid after the tables were rebuilt for the second.
"""
import numpy as np
import pytest
import torch

import paper_2010_04760_amd as T
import workloads as W
from paper_2010_04760_amd import _binding as B

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def _case(nr, nth, s, m, a, wp, seed, order=2):
    wl = W.C2.with_(nr=nr, nth=nth, s=s, m=m, a=a, seed=seed, x_min=-100.0, x_max=200.0)
    probe = T.make_config(s=wl.s, m=wl.m, a=wl.a, nr=wl.nr, ntheta=wl.nth, x_min=wl.x_min, x_max=wl.x_max,
                          weight_prec=wp, theta_order=order)
    with T.Solver(probe) as sv:
        dt = sv.info().dt
    cfg = T.make_config(s=wl.s, m=wl.m, a=wl.a, nr=wl.nr, ntheta=wl.nth, x_min=wl.x_min, x_max=wl.x_max,
                        weight_prec=wp, dt=dt, theta_order=order)
    return wl, cfg


def _reference(cfg, u0, nsteps):
    with T.Solver(cfg) as sv:
        sv.set_initial(u0)
        sv.step(nsteps)
        return sv.state()


def _noalloc(cfg, u0, nsteps):
    u = torch.from_numpy(np.ascontiguousarray(u0)).to("cuda")
    T.teuk_step_noalloc(cfg, u, nsteps)
    torch.cuda.synchronize()
    return u.cpu().numpy()


@pytest.mark.parametrize("wp,order", [("fp64", 2), ("fp32", 2), ("fp64", 4)])
def test_noalloc_equals_teuk_step_two_calls_second_smaller(wp, order):
    cases = [(1000, 96, -2, 2, 0.999, 11, 40), (300, 20, 0, 0, 0.5, 12, 25), (1000, 96, -2, 2, 0.999, 13, 10)]
    for nr, nth, s, m, a, seed, nsteps in cases:
        wl, cfg = _case(nr, nth, s, m, a, wp, seed, order)
        u0 = W.gaussian_pulse(wl)
        say(f"noalloc {wp} theta order {order}: {nr}x{nth} s={s} m={m} a={a} seed={seed}, {nsteps} steps")
        ref = _reference(cfg, u0, nsteps)
        got = _noalloc(cfg, u0, nsteps)
        assert np.all(np.isfinite(got))
        assert np.max(np.abs(got - u0.reshape(got.shape))) > 0      # the state did advance
        np.testing.assert_array_equal(got, ref)


def test_noalloc_rejects_what_it_cannot_hold():
    u = torch.zeros(4 * 64 * 64, dtype=torch.float64, device="cuda")
    base = dict(s=0, m=0, a=0.5, x_min=-50.0, x_max=50.0, dt=0.01)
    too_big = T.make_config(nr=32768, ntheta=64, **base)                  # 2^21 points > 2^20
    with pytest.raises(T.TeukError) as ei:
        B._check(B._lib.teuk_step_noalloc(ctypes_cfg(too_big), ctypes_ptr(u), 1, None))
    assert ei.value.status == T.TEUK_ERR_INVALID_ARG and "scratch limits" in str(ei.value)
    no_dt = T.make_config(nr=64, ntheta=64, **{**base, "dt": 0.0})
    with pytest.raises(T.TeukError) as ei:
        T.teuk_step_noalloc(no_dt, u, 1)
    assert ei.value.status == T.TEUK_ERR_INVALID_ARG
    chart_h = T.make_config(nr=64, ntheta=64, s=-2, m=0, a=1.0, x_min=20.0 / 21.0, x_max=19.0, chart="H", dt=0.01)
    with pytest.raises(T.TeukError) as ei:
        T.teuk_step_noalloc(chart_h, u, 1)
    assert ei.value.status == T.TEUK_ERR_UNSUPPORTED
    # nothing was enqueued by the failed calls: the state is untouched
    torch.cuda.synchronize()
    assert float(u.abs().max()) == 0.0


def ctypes_cfg(cfg):
    import ctypes
    return ctypes.byref(cfg)


def ctypes_ptr(t):
    import ctypes
    return ctypes.c_void_p(t.data_ptr())
