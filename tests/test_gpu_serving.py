"""GPU: the continuous-batching server.

Small requests of uneven size arrive over time; the server admits them by
HBM footprint, steps them together in chunks and returns each waveform.  Each
served result must equal the same request run alone (teuk_step) bit for bit,
whatever the mix it was stepped in; a tight HBM budget must bound the resident
set; a request larger than the budget is rejected."""
import numpy as np
import pytest

import paper_2010_04760_amd as T
import workloads as W
from paper_2010_04760_amd import serving

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def small_requests(n, seed=3, grid=None):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        nr, nth = grid if grid else (int(rng.integers(64, 400)), int(rng.integers(4, 24)))
        wl = W.Workload(f"small[{i}]", s=int(rng.choice([0, -2])), m=int(rng.integers(0, 5)),
                        a=float(rng.uniform(0.5, 1.0)), nr=nr, nth=nth, x_min=-40.0, x_max=60.0,
                        steps=int(rng.integers(10, 60)), seed=500 + i, every=3)
        out.append(serving.Request(i, wl, weights=["fp64", "fp32"][i % 2]))
    return out


def alone(req):
    with T.Solver(req.config()) as sv:
        sv.set_initial(W.gaussian_pulse(req.wl))
        sv.step(req.steps)
        t, w = sv.waveform()
        return t, w, sv.state()


def check_identical(res, reqs):
    assert len(res.done) == len(reqs)
    for d in res.done:
        t, w, st = alone(d.req)
        assert np.array_equal(d.times, t), d.req.rid
        assert np.array_equal(d.waveform, w), d.req.rid
        assert np.array_equal(d.state, st), d.req.rid
        assert d.finished >= d.admitted >= d.arrival - 1e-9


def test_served_equals_alone():
    reqs = small_requests(10)
    arrivals = np.concatenate([np.zeros(5), np.linspace(0.01, 0.05, len(reqs) - 5)])
    say("case serving: 10 requests, chunk 7")
    res = serving.Server(max_members=16, chunk_steps=7, keep_state=True).run(reqs, arrivals)
    assert res.max_resident >= 2            # some requests did share launches
    check_identical(res, reqs)


def test_budget_bounds_resident_set():
    reqs = small_requests(6, seed=4, grid=(300, 12))     # equal footprints (equal step counts aside)
    fps = [T.teuk_footprint_bytes(r.config()) for r in reqs]
    budget = 2 * max(fps) + min(fps) // 2                # two fit, three do not
    big = W.Workload("too big", s=0, m=0, a=0.5, nr=4096, nth=64, x_min=-40.0, x_max=60.0, steps=5, seed=9)
    reqs_all = reqs + [serving.Request(99, big)]
    say("case serving budget", budget)
    res = serving.Server(max_members=8, hbm_budget=budget, chunk_steps=5, keep_state=True).run(
        reqs_all, np.zeros(len(reqs_all)))
    assert [r.rid for r in res.rejected] == [99]
    assert 1 <= res.max_resident <= 2
    check_identical(res, reqs)
