"""GPU: the group extension (many independent solves, one launch per RK stage
for each cache block of members).

A member's arithmetic is the single-solve stage arithmetic, tile by tile, so a
solve advanced inside a group must equal the same solve advanced alone bit for
bit: state, waveform samples and counters.  Cases: a mixed group (ragged grids,
different spins, Kerr parameters, weight precisions, sampling intervals and
tile sizes), members joining and leaving mid-run, members cut into several
cache blocks, members of both charts, the batched workload mix at full size
(several members checked), one member against the FP64 oracle, and the error
paths."""
import numpy as np
import pytest
import torch

import paper_2010_04760_amd as T
import workloads as W
from oracle import solver as S

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


MIX = [  # nr, nth, s, m, a, weights, every
    (7, 2, 0, 0, 0.5, "fp64", 1),
    (63, 5, -2, 2, 0.999, "fp64", 2),
    (200, 17, -2, 1, 1.0, "fp32", 3),
    (513, 33, 0, 2, 0.7, "fp64", 0),
    (127, 64, -2, 3, 0.9, "fp16", 5),
    (300, 40, 0, 0, 0.0, "bf16", 1),
    (1000, 19, -2, 4, 0.6, "fp32", 4),
]


def make(nr, nth, s, m, a, weights, every, seed):
    cfg = T.make_config(s=s, m=m, a=a, nr=nr, ntheta=nth, x_min=-30.0, x_max=50.0, weight_prec=weights,
                        x_extract=10.0, extract_every=every, max_samples=64 if every else 0)
    sv = T.Solver(cfg)
    u0 = W.random_state(nr, nth, seed=seed, smooth=True)
    sv.set_initial(u0)
    return sv, u0


def snapshot(sv):
    st = sv.state()
    t, w = sv.waveform() if sv.cfg.extract_every else (np.zeros(0), np.zeros(0))
    inf = sv.info()
    return st, t, w, (inf.steps, inf.samples, inf.t)


def assert_same(a, b, what):
    for x, y in zip(a[:3], b[:3]):
        assert x.shape == y.shape, what
        assert np.array_equal(x, y), (what, float(np.max(np.abs(x - y))) if x.size else 0.0)
    assert a[3] == b[3], (what, a[3], b[3])


@pytest.mark.parametrize("wg,rows", [(0, 0), (1, 3), (7, 1), (64, 5), (100000, 16), (0, 1000)])
def test_group_equals_alone_bitwise(wg, rows):
    say("case group mix, workgroups", wg, "rows per tile", rows)
    nsteps = 7
    alone = []
    for i, spec in enumerate(MIX):
        sv, _ = make(*spec, seed=100 + i)
        sv.step(nsteps)
        alone.append(snapshot(sv))
        sv.close()
    members = [make(*spec, seed=100 + i)[0] for i, spec in enumerate(MIX)]
    with T.Group(len(MIX), workgroups=wg, rows_per_tile=rows) as g:
        for sv in members:
            g.add(sv)
        inf = g.info()
        assert inf.members == len(MIX) and inf.classes == 4
        assert inf.points == sum(s[0] * s[1] for s in MIX)
        assert inf.units == sum(-(-s[0] // 63) * s[1] for s in MIX)
        assert inf.workgroups >= 4 and (wg == 0 or inf.workgroups <= 4 * wg)
        assert inf.workgroups <= inf.tiles
        g.step(3)
        g.step(0)
        g.step(nsteps - 3)
        for i, sv in enumerate(members):
            assert_same(snapshot(sv), alone[i], MIX[i])
    for sv in members:
        sv.close()


def test_members_join_and_leave():
    say("case join/leave")
    specs = MIX[1:4]
    # reference: each solve alone for its total step count
    plan = {0: 9, 1: 9, 2: 9}
    ref = []
    for i, spec in enumerate(specs):
        sv, _ = make(*spec, seed=200 + i)
        sv.step(plan[i])
        ref.append(snapshot(sv))
        sv.close()
    a, _ = make(*specs[0], seed=200)
    b, _ = make(*specs[1], seed=201)
    c, _ = make(*specs[2], seed=202)
    with T.Group(4) as g:
        g.add(a)
        g.step(2)              # a: 2
        g.add(b)
        b.step(1)              # b alone: 1 (same stream, allowed between group steps)
        g.step(3)              # a: 5, b: 4
        g.remove(a)
        a.step(4)              # a alone: 9
        g.add(c)
        g.step(5)              # b: 9, c: 5
        g.remove(b)
        g.step(4)              # c: 9
        assert g.info().members == 1
    for i, sv in enumerate((a, b, c)):
        assert_same(snapshot(sv), ref[i], ("join/leave", i))
        sv.close()


def test_member_against_oracle():
    say("case group member vs oracle")
    prob = S.Problem(-2, 2, 0.999, 190, 24, -30.0, 50.0)
    o = S.TeukOracle(prob)
    dt = 0.4 * o.dt_bound(1.0)
    u0 = W.random_state(prob.nr, prob.nth, seed=7, smooth=True)
    ref, _ = o.evolve(u0, dt, 5)
    cfg = T.make_config(s=prob.s, m=prob.m, a=prob.a, nr=prob.nr, ntheta=prob.nth, x_min=prob.x_min,
                        x_max=prob.x_max, dt=dt)
    other, _ = make(*MIX[2], seed=5)
    with T.Solver(cfg) as sv, T.Group(2) as g:
        sv.set_initial(u0)
        g.add(other)
        g.add(sv)
        g.step(5)
        got = sv.state()
    other.close()
    err = float(np.max(np.abs(got - ref))) / float(np.max(np.abs(ref)))
    say("  state error", err)
    assert err <= 1e-12


def test_cache_blocks_bitwise():
    """Members large enough that the group cuts them into several cache blocks
    (footprints of about 100 MB against 256 MiB per block), in two precision
    classes with different sampling intervals: every member, stepped by the
    group in two calls, equals the same solve alone, bitwise."""
    say("case group cache blocks")
    spec = [(8192, 128, -2, 2, 0.999, "fp64", 2), (8192, 128, 0, 1, 0.7, "fp32", 3),
            (8000, 130, -2, 0, 0.5, "fp64", 1), (8192, 120, 0, 3, 0.9, "fp32", 0),
            (8100, 128, -2, 1, 1.0, "fp64", 4), (7000, 140, 0, 0, 0.6, "fp64", 2)]
    members = [make(*sp, seed=70 + i) for i, sp in enumerate(spec)]
    fp64_bytes = sum(T.teuk_footprint_bytes(sv.cfg) for (sv, _), sp in zip(members, spec) if sp[5] == "fp64")
    assert fp64_bytes > 256 << 20          # the FP64 class spans more than one block
    with T.Group(len(spec)) as g:
        for sv, _ in members:
            g.add(sv)
        g.step(2)
        g.step(3)
        torch.cuda.synchronize()
        got = [snapshot(sv) for sv, _ in members]
    say("   FP64 class footprint", fp64_bytes >> 20, "MiB")
    for (sv, u0), sp, gs in zip(members, spec, got):
        sv.close()
        alone, _ = make(*sp, seed=0)
        alone.set_initial(u0)
        alone.step(5)
        assert_same(gs, snapshot(alone), ("member", sp))
        alone.close()


def test_group_with_hyperboloidal_members():
    """Members of both charts in one group (tortoise FP64 and FP32, hyperboloidal
    FP64 and FP16, a = M with the grid starting on the horizon and a = 0.8 with
    it inside): state, waveform, horizon samples and counters equal each solve
    alone, bitwise."""
    say("case group with chart-H members")

    def make_h(nr, nth, a, x_min, weights, every, seed):
        cfg = T.make_config(s=-2, m=0, a=a, nr=nr, ntheta=nth, x_min=x_min, x_max=19.5, chart="H", S=20.0,
                            weight_prec=weights, x_extract=19.0, extract_every=every, max_samples=16)
        sv = T.Solver(cfg)
        u0 = W.random_state(nr, nth, seed=seed, smooth=True)
        sv.set_initial(u0)
        return sv, u0

    spec_h = [(300, 12, 1.0, 20.0 / 21.0, "fp64", 2), (257, 9, 0.8, 1.2, "fp16", 3)]
    spec_t = [(200, 17, -2, 1, 1.0, "fp64", 1), (513, 8, 0, 2, 0.7, "fp32", 2)]
    hmem = [make_h(*sp, seed=90 + i) for i, sp in enumerate(spec_h)]
    tmem = [make(*sp, seed=95 + i) for i, sp in enumerate(spec_t)]
    with T.Group(4) as g:
        for sv, _ in hmem + tmem:
            g.add(sv)
        assert g.info().classes == 4
        g.step(4)
        g.step(3)
        torch.cuda.synchronize()
        got_h = [(snapshot(sv), sv.horizon()) for sv, _ in hmem]
        got_t = [snapshot(sv) for sv, _ in tmem]
    for (sv, u0), sp, (gs, gh) in zip(hmem, spec_h, got_h):
        sv.close()
        alone, _ = make_h(*sp, seed=0)
        alone.set_initial(u0)
        alone.step(7)
        assert_same(gs, snapshot(alone), ("chart H member", sp))
        for x, y in zip(gh, alone.horizon()):
            assert np.array_equal(x, y), ("horizon samples", sp)
        alone.close()
    for (sv, u0), sp, gs in zip(tmem, spec_t, got_t):
        sv.close()
        alone, _ = make(*sp, seed=0)
        alone.set_initial(u0)
        alone.step(7)
        assert_same(gs, snapshot(alone), ("chart T member", sp))
        alone.close()


def test_batched_mix_full_size():
    """The 64-solve mix at full size, 2 steps in one group; four members (the
    largest, the smallest and two others) against the same solves alone."""
    mix = W.batch_workloads()
    say("case batched mix full size:", len(mix), "solves,", sum(w.points for w in mix), "points")
    members = []
    for w in mix:
        cfg = T.make_config(s=w.s, m=w.m, a=w.a, nr=w.nr, ntheta=w.nth, x_min=w.x_min, x_max=w.x_max,
                            weight_prec="fp32", x_extract=w.x_e, extract_every=1, max_samples=4)
        sv = T.Solver(cfg)
        sv.set_initial(W.gaussian_pulse(w))
        members.append(sv)
    with T.Group(len(mix)) as g:
        for sv in members:
            g.add(sv)
        g.step(2)
        torch.cuda.synchronize()
        sizes = [w.points for w in mix]
        pick = sorted({int(np.argmax(sizes)), int(np.argmin(sizes)), 17, 42})
        got = {i: snapshot(members[i]) for i in pick}
    for sv in members:
        sv.close()
    for i in pick:
        w = mix[i]
        cfg = T.make_config(s=w.s, m=w.m, a=w.a, nr=w.nr, ntheta=w.nth, x_min=w.x_min, x_max=w.x_max,
                            weight_prec="fp32", x_extract=w.x_e, extract_every=1, max_samples=4)
        with T.Solver(cfg) as sv:
            sv.set_initial(W.gaussian_pulse(w))
            sv.step(2)
            assert_same(got[i], snapshot(sv), ("mix member", i, w.nr, w.nth))


def test_group_errors():
    say("case group errors")
    with pytest.raises(T.TeukError) as ei:
        T.teuk_group_create(None, 0)
    assert ei.value.status == T.TEUK_ERR_INVALID_ARG
    cfg = T.make_config(s=0, m=0, a=0.5, nr=64, ntheta=4, x_min=-10, x_max=10)
    with T.Group(1) as g:
        fresh = T.Solver(cfg)
        with pytest.raises(T.TeukError) as ei:
            g.add(fresh)                       # no initial data
        assert ei.value.status == T.TEUK_ERR_STATE
        fresh.set_initial(W.random_state(64, 4, seed=1))
        g.add(fresh)
        with pytest.raises(T.TeukError) as ei:
            g.add(fresh)                       # already a member
        assert ei.value.status == T.TEUK_ERR_INVALID_ARG
        other = T.Solver(cfg)
        other.set_initial(W.random_state(64, 4, seed=2))
        with pytest.raises(T.TeukError) as ei:
            g.add(other)                       # group full
        assert ei.value.status == T.TEUK_ERR_CAPACITY
        side = torch.cuda.Stream()
        sv_side = T.Solver(cfg, stream=side)
        sv_side.set_initial(W.random_state(64, 4, seed=3))
        g.remove(fresh)
        with pytest.raises(T.TeukError) as ei:
            g.add(sv_side)                     # other stream
        assert ei.value.status == T.TEUK_ERR_INVALID_ARG
        with pytest.raises(T.TeukError) as ei:
            g.remove(other)                    # not a member
        assert ei.value.status == T.TEUK_ERR_INVALID_ARG
        with pytest.raises(T.TeukError) as ei:
            g.step(-1)
        assert ei.value.status == T.TEUK_ERR_INVALID_ARG
        g.add(other)
        other.close()                          # destroying a member detaches it
        assert g.info().members == 0
        g.step(2)                              # empty group: no-op
        for sv in (fresh, sv_side):
            sv.close()


@pytest.mark.parametrize("chunk", [0, 4])
def test_blocked_members_bitwise(chunk):
    """Members with the temporally blocked step (FP64 and FP32 weights) beside
    three-launch members: each blocked member is a cache block of its own,
    stepped by its own blocked launches (which trade its two state buffers
    every step), so the group must still equal every member stepped alone,
    eagerly and in graph mode (an even chunk; an odd one is refused)."""
    say("case group with blocked members, graph chunk", chunk)
    # sampling intervals of 1 and 0, so that only the buffer swaps forbid an odd chunk
    specs = [(300, 17, -2, 1, 1.0, "fp32", 1, "rk3_blocked"), (200, 9, 0, 2, 0.7, "fp64", 1, "rk3"),
             (513, 12, -2, 2, 0.999, "fp64", 0, "rk3_blocked"), (130, 33, 0, 0, 0.5, "fp32", 0, "rk3")]
    alone, members = [], []
    g = T.Group(len(specs))
    for i, (nr, nth, s_, m, a, wp, every, integ) in enumerate(specs):
        cfg = T.make_config(s=s_, m=m, a=a, nr=nr, ntheta=nth, x_min=-30.0, x_max=50.0, weight_prec=wp,
                            x_extract=10.0, extract_every=every, max_samples=64 if every else 0, integrator=integ)
        u0 = W.random_state(nr, nth, seed=70 + i, smooth=True)
        ref = T.Solver(cfg)
        ref.set_initial(u0)
        for n in (3, 8, 5):
            ref.step(n)
        alone.append(snapshot(ref))
        ref.close()
        sv = T.Solver(cfg)
        sv.set_initial(u0)
        g.add(sv)
        members.append(sv)
    if chunk:
        with pytest.raises(T.TeukError) as ei:
            g.set_graph(chunk + 1)
        assert ei.value.status == T.TEUK_ERR_INVALID_ARG
        g.set_graph(chunk)
    for n in (3, 8, 5):
        g.step(n)
    for i, sv in enumerate(members):
        assert_same(snapshot(sv), alone[i], ("blocked member", i, chunk))
    g.close()
    for sv in members:
        sv.close()


@pytest.mark.parametrize("chunk", [0, 6])
def test_solo_blocks_bitwise(chunk):
    """Members that each fill the GPU (strips x rows above the resident
    workgroups) form solo cache blocks, stepped by their own single-solve
    launches member after member: the group must still equal every member
    stepped alone, eagerly and from captured graphs, and report the members'
    own launch shapes.  With the batched launch's workgroup count fixed by the
    caller the same members take the batched launch, with the same results."""
    say("case solo cache blocks, graph chunk", chunk)
    specs = [(4096, 72, -2, 2, 0.9, "fp64", 3, 2), (4200, 70, 0, 1, 0.6, "fp32", 2, 2),
             (4150, 66, -2, 0, 0.99, "fp64", 0, 2), (4100, 68, -2, 1, 0.8, "fp64", 1, 4)]
    alone, cfgs, u0s = [], [], []
    for i, (nr, nth, s_, m, a, wp, every, order) in enumerate(specs):
        cfg = T.make_config(s=s_, m=m, a=a, nr=nr, ntheta=nth, x_min=-100.0, x_max=300.0, weight_prec=wp,
                            x_extract=30.0, extract_every=every, max_samples=64 if every else 0, theta_order=order)
        u0 = W.random_state(nr, nth, seed=90 + i, smooth=True)
        with T.Solver(cfg) as ref:
            ref.set_initial(u0)
            for n in (4, 12, 7):
                ref.step(n)
            alone.append(snapshot(ref))
            own_wg = ref.info().workgroups
        cfgs.append(cfg)
        u0s.append(u0)
    for wg in (0, 1000):
        members = []
        g = T.Group(len(specs), workgroups=wg)
        for cfg, u0 in zip(cfgs, u0s):
            sv = T.Solver(cfg)
            sv.set_initial(u0)
            g.add(sv)
            members.append(sv)
        inf = g.info()
        if wg == 0:
            # the two second-order FP64 members (about 28 MB each) share one solo block, the FP32 and
            # the fourth-order members have their own; each is launched with its own tiling, so the
            # reported workgroups equal the tiles
            assert inf.workgroups == inf.tiles
        if chunk:
            g.set_graph(chunk)
        for n in (4, 12, 7):
            g.step(n)
        for i, sv in enumerate(members):
            assert_same(snapshot(sv), alone[i], ("solo block member", i, wg, chunk))
        g.close()
        for sv in members:
            sv.close()
