"""Host-side checks of the C ABI (no GPU needed): the library loads and exports
every entry point include/teuk.h declares, the ctypes structures match the C
layout, the host tables and per-point coefficient formula agree with the
oracle's symbolic derivation, and invalid configurations are rejected."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import paper_2010_04760_amd as T
from oracle import solver as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "teuk.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(teuk_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    lib = ctypes.CDLL(T.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(T.EXPORTED) == names


def test_struct_layout_matches_c(tmp_path):
    probe = tmp_path / "probe.c"
    probe.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "teuk.h"
#define F(s, f) printf(#s "." #f " %zu\\n", offsetof(s, f));
int main(void) {
  printf("teuk_config %zu\\n", sizeof(teuk_config));
  printf("teuk_device_ctx %zu\\n", sizeof(teuk_device_ctx));
  printf("teuk_info_t %zu\\n", sizeof(teuk_info_t));
  printf("teuk_group_info_t %zu\\n", sizeof(teuk_group_info_t));
  printf("teuk_tune_info_t %zu\\n", sizeof(teuk_tune_info_t));
  printf("teuk_group_tune_info_t %zu\\n", sizeof(teuk_group_tune_info_t));
  F(teuk_config, M) F(teuk_config, a) F(teuk_config, x_extract) F(teuk_config, workgroups) F(teuk_config, S)
  F(teuk_config, state_prec) F(teuk_config, integrator) F(teuk_config, scheme) F(teuk_config, ko_sigma)
  F(teuk_info_t, samples) F(teuk_info_t, dt_bound) F(teuk_device_ctx, workspace_bytes)
  F(teuk_group_info_t, workgroups) F(teuk_group_info_t, points)
  F(teuk_tune_info_t, steps) F(teuk_tune_info_t, us_per_step) F(teuk_tune_info_t, us_per_step_default)
  F(teuk_group_tune_info_t, steps) F(teuk_group_tune_info_t, us_per_step) F(teuk_group_tune_info_t, us_per_step_default)
  return 0; }
""")
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(probe), "-o", str(exe)], check=True)
    out = dict(line.rsplit(" ", 1) for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                                check=True).stdout.split("\n") if line)
    assert int(out["teuk_config"]) == ctypes.sizeof(T.teuk_config)
    assert int(out["teuk_device_ctx"]) == ctypes.sizeof(T.teuk_device_ctx)
    assert int(out["teuk_info_t"]) == ctypes.sizeof(T.teuk_info_t)
    for st in ("teuk_group_info_t", "teuk_tune_info_t", "teuk_group_tune_info_t"):
        assert int(out[st]) == ctypes.sizeof(getattr(T, st)), st
    for key, val in out.items():
        if "." in key:
            s, f = key.split(".")
            assert getattr(getattr(T, s), f).offset == int(val), key


CASES = [(0, 0, 0.5, -64.0, 64.0), (-2, 2, 0.999, -200.0, 400.0), (0, 0, 1.0, -400.0, 800.0),
         (-2, 4, 1.0, -100.0, 300.0), (1, -3, 0.3, -50.0, 60.0), (-2, 1, 0.0, -300.0, 300.0)]
NAMES = ["lam1", "m3r", "m3i", "btr", "bti", "cr", "ci", "ath", "bth", "lam2"]


@pytest.mark.parametrize("s,m,a,x0,x1", CASES)
def test_host_coefficients_match_oracle(s, m, a, x0, x1):
    nr, nth = 301, 12
    cfg = T.make_config(s=s, m=m, a=a, nr=nr, ntheta=nth, x_min=x0, x_max=x1)
    hc = T.teuk_host_coefficients(cfg)
    o = S.TeukOracle(S.Problem(s, m, a, nr, nth, x0, x1))
    scale = max(np.max(np.abs(o.tab[n])) for n in NAMES)
    for i, n in enumerate(NAMES):
        ref = o.tab[n]
        err = np.max(np.abs(hc[i] - ref))
        assert err <= 1e-13 * np.max(np.abs(ref)) + 1e-15 * scale, (n, err, np.max(np.abs(ref)))
    np.testing.assert_allclose(o.tab["lam2"], -hc[0], rtol=1e-14)


def chart_h_grid(a, nr, S=20.0, lo=0.55, hi_gap=0.3):
    """x_min, x_max of a chart-H grid from lo * rho_H to S - hi_gap, nudged so
    that no node falls on the horizon."""
    rp, _ = S_oracle_horizons(a)
    rho_h = S * rp / (rp + S)
    x0, x1 = lo * rho_h, S - hi_gap
    dx = (x1 - x0) / (nr - 1)
    f = (rho_h - x0) / dx
    if abs(f - round(f)) < 0.05:
        x0 -= 0.3 * dx
        x1 -= 0.3 * dx
    return x0, x1


def S_oracle_horizons(a):
    from oracle import coefficients as C
    return C.horizons(1.0, a)


CASES_H = [(-2, 0, 1.0), (-2, 2, 0.999), (0, 1, 0.5), (0, 0, 0.0), (1, -3, 0.8)]


@pytest.mark.parametrize("s,m,a", CASES_H)
def test_host_coefficients_match_oracle_chart_H(s, m, a):
    nr, nth = 157, 8
    x0, x1 = chart_h_grid(a, nr)
    cfg = T.make_config(s=s, m=m, a=a, nr=nr, ntheta=nth, x_min=x0, x_max=x1, chart="H", S=20.0)
    hc = T.teuk_host_coefficients(cfg)
    o = S.TeukOracle(S.Problem(s, m, a, nr, nth, x0, x1, chart="H", S=20.0))
    scale = max(np.max(np.abs(o.tab[n])) for n in NAMES)
    for i, n in enumerate(NAMES):
        ref = o.tab[n]
        err = np.max(np.abs(hc[i] - ref))
        assert err <= 1e-13 * np.max(np.abs(ref)) + 1e-15 * scale, (n, err, np.max(np.abs(ref)))


def test_chart_H_validation():
    a = 1.0
    x0, x1 = chart_h_grid(a, 101)
    ok = T.make_config(s=-2, m=0, a=a, nr=101, ntheta=8, x_min=x0, x_max=x1, chart="H", S=20.0)
    assert T.teuk_footprint_bytes(ok) > 0
    # a grid that starts on the horizon is admissible (one-sided horizon stencil)
    on = T.make_config(s=-2, m=0, a=a, nr=101, ntheta=8, x_min=20.0 / 21.0, x_max=x1, chart="H", S=20.0)
    assert T.teuk_footprint_bytes(on) > 0
    rp, _ = S_oracle_horizons(a)
    rho_h = 20.0 * rp / (rp + 20.0)
    bad = [
        dict(x_min=x0, x_max=20.0),                 # reaches S
        dict(x_min=0.0, x_max=x1),                  # r = 0
        dict(x_min=rho_h + 0.5, x_max=x1),          # horizon more than half a step below the grid
        dict(x_min=x0, x_max=x1, S=-1.0),
    ]
    for kw in bad:
        args = dict(s=-2, m=0, a=a, nr=101, ntheta=8, chart="H", S=20.0)
        args.update(kw)
        c = T.make_config(**args)
        assert T.teuk_footprint_bytes(c) == 0, kw


def test_footprint_and_validation():
    ok = T.make_config(s=0, m=0, a=0.5, nr=512, ntheta=32, x_min=-64, x_max=64)
    fp = T.teuk_footprint_bytes(ok)
    assert fp >= 3 * 4 * 512 * 32 * 8
    bad = []
    for field, val in [("a", 1.5), ("nr", 6), ("ntheta", 1), ("weight_prec", 7), ("abi_version", 99),
                       ("chart", 3), ("weno_eps", 0.0), ("M", -1.0), ("s", 3), ("theta_order", 3),
                       ("theta_order", 6)]:
        c = T.make_config(s=0, m=0, a=0.5, nr=512, ntheta=32, x_min=-64, x_max=64)
        setattr(c, field, val)
        bad.append(c)
    c = T.make_config(s=0, m=0, a=0.5, nr=512, ntheta=32, x_min=64, x_max=-64)
    bad.append(c)
    c = T.make_config(s=0, m=0, a=0.5, nr=512, ntheta=32, x_min=-64, x_max=64, extract_every=5, max_samples=0)
    bad.append(c)
    c = T.make_config(s=0, m=0, a=0.5, nr=512, ntheta=32, x_min=-64, x_max=64, extract_every=5, max_samples=3,
                      x_extract=100.0)
    bad.append(c)
    for c in bad:
        assert T.teuk_footprint_bytes(c) == 0
        with pytest.raises(T.TeukError) as ei:
            T.teuk_host_coefficients(c)
        assert ei.value.status == T.TEUK_ERR_INVALID_ARG
        assert T.teuk_last_error(None)


def test_theta_order_field():
    d = T.teuk_default_config()
    assert d.theta_order == 2
    for order in (0, 2, 4):
        c = T.make_config(s=-2, m=2, a=0.9, nr=512, ntheta=32, x_min=-64, x_max=64, theta_order=order)
        assert T.teuk_footprint_bytes(c) > 0, order


def test_capacity_error():
    cfg = T.make_config(s=0, m=0, a=0.5, nr=64, ntheta=4, x_min=-10, x_max=10)
    lib = ctypes.CDLL(T.LIB_PATH)
    lib.teuk_host_coefficients.argtypes = [ctypes.POINTER(T.teuk_config), ctypes.POINTER(ctypes.c_double),
                                           ctypes.c_size_t]
    out = np.zeros(10)
    st = lib.teuk_host_coefficients(ctypes.byref(cfg), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 10)
    assert st == T.TEUK_ERR_CAPACITY
    st = lib.teuk_host_coefficients(ctypes.byref(cfg), None, 10**6)
    assert st == T.TEUK_ERR_INVALID_ARG


def test_too_deep_horizon_is_rejected():
    # a = 0, x_min = -1600: Delta ~ exp(-800) underflows FP64
    cfg = T.make_config(s=0, m=0, a=0.0, nr=64, ntheta=4, x_min=-1600.0, x_max=10.0)
    with pytest.raises(T.TeukError) as ei:
        T.teuk_host_coefficients(cfg)
    assert ei.value.status == T.TEUK_ERR_INVALID_ARG


def test_destroy_null_is_safe():
    T.teuk_destroy(None)
