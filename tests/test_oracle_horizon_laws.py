"""Oracle pin: the horizon laws of paper Sec. 4 on extremal Kerr.

Sec. 4 evolves s = -2 axisymmetric data in the hyperboloidal chart with the
horizon of an a = M hole on the grid and finds, on the horizon, the field
decaying as 1/tau while its radial derivative tends to a non-zero constant
(the Aretakis behaviour).  The oracle's runs of that experiment on radial
grids of 512 to 4096 points are stored in tests/golden/horizon_series.txt by
tests/golden/make_horizon_series.py, which calls only the oracle (about
16 minutes on 8 cores).

This test first ties the stored series to the oracle as it stands: it reruns
the 512-point series in full and the first samples of the three finer ones,
which must agree with the file.  It then checks the laws on the stored series:

* d_rho Phi_H: its local index over tau in [250, 500] halves with every halving
  of the radial step (first-order convergence to 0), is below 0.02 on the
  finest grid, and its two-grid extrapolation is 0 within 0.05; the value at
  tau = 500 settles at a non-zero constant;
* Phi_H: the end-value closure of the inner edge leaves a floor of first
  order in the radial step (the late value halves with the step); the
  three-grid Richardson value, which removes the O(dx) and O(dx^2) parts,
  has local index -1 within 0.05 over tau in [30, 100], where tau Phi_H stays
  constant within 5 %.

A mistake in the chart-H evolution (coefficients, the sign of a speed, the
upwind side, the inner-edge closure, the sampler) changes the series, so
either the rerun no longer matches the file or, once the file is rewritten by
the generator, the laws fail.
"""
import importlib.util
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden", "horizon_series.txt")


def _generator():
    spec = importlib.util.spec_from_file_location("_make_horizon_series",
                                                  os.path.join(ROOT, "tests", "golden", "make_horizon_series.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _load():
    grids, cur = {}, None
    with open(GOLDEN) as f:
        for ln in f:
            if ln.startswith("#"):
                continue
            p = ln.split()
            if p[0] == "grid":
                cur = int(p[1])
                grids[cur] = {"dt": float(p[3]), "every": int(p[5]), "rows": []}
            else:
                grids[cur]["rows"].append([float(x) for x in p])
    for g in grids.values():
        g["rows"] = np.array(g["rows"])
    return grids


def local_index(t, y):
    """p(t) = t (dy/dt) / y by centred differences (the paper's local power-law index)."""
    return t[1:-1] * (y[2:] - y[:-2]) / (t[2:] - t[:-2]) / y[1:-1]


@pytest.fixture(scope="module")
def series():
    return _load()


def test_stored_series_come_from_this_oracle(series):
    gen = _generator()
    from oracle import solver as S
    S.set_threads(os.cpu_count() or 1)
    for nr, nsamp in ((512, None), (1024, 4), (2048, 3), (4096, 2)):
        dt, every, t, ph, dph = gen.series(nr, max_samples=nsamp)
        ref = series[nr]["rows"]
        assert dt == series[nr]["dt"] and every == series[nr]["every"], nr
        n = len(t)
        assert n == (len(ref) if nsamp is None else nsamp + 1), nr
        np.testing.assert_allclose(t, ref[:n, 0], rtol=0, atol=1e-12)
        for col, live in ((1, ph), (2, dph)):
            scale = np.max(np.abs(ref[:n, col]))
            assert np.max(np.abs(live - ref[:n, col])) <= 1e-12 * scale, (nr, col)


def test_horizon_derivative_tends_to_a_constant(series):
    idx = {}
    for nr, g in series.items():
        t, dph = g["rows"][:, 0], g["rows"][:, 2]
        late = t[1:-1] >= 250.0
        idx[nr] = float(np.mean(local_index(t, dph)[late]))
    # first-order convergence of the late index to 0
    for c, f in ((512, 1024), (1024, 2048)):
        assert 0.0 < idx[f] < idx[c]
        assert 1.7 < idx[c] / idx[f] < 2.5, (c, f, idx)
    assert abs(idx[4096]) < 0.02, idx
    assert abs(2.0 * idx[4096] - idx[2048]) < 0.05, idx
    # the limit is a non-zero constant
    end = {nr: g["rows"][-1, 2] for nr, g in series.items()}
    assert end[4096] > 1.0
    assert abs(end[4096] - end[2048]) < 0.03 * end[4096], end


def test_horizon_field_decays_as_one_over_tau(series):
    # the first-order floor of the inner-edge closure: the late value halves
    # with the radial step
    late = {nr: g["rows"][-1, 1] for nr, g in series.items()}
    for c, f in ((1024, 2048), (2048, 4096)):
        assert 1.8 < late[c] / late[f] < 2.4, late
    # three-grid Richardson value on tau in [30, 100]
    tau = np.linspace(30.0, 100.0, 141)
    y = {nr: np.interp(tau, series[nr]["rows"][:, 0], series[nr]["rows"][:, 1]) for nr in (1024, 2048, 4096)}
    rich = (8.0 * y[4096] - 6.0 * y[2048] + y[1024]) / 3.0
    p = local_index(tau, rich)
    assert abs(float(np.mean(p)) + 1.0) < 0.05, float(np.mean(p))
    tphi = tau * rich
    assert (tphi.max() - tphi.min()) < 0.05 * abs(tphi.mean()), (tphi.min(), tphi.max())
