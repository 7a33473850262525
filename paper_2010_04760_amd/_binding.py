"""ctypes binding of libteuk (include/teuk.h): argument marshalling only.

Every computation runs in the HIP library.  PyTorch supplies device memory
(a workspace tensor the solver lives in) and streams; it is imported before
the library is loaded so that both share one HIP runtime.  If libteuk.so is
not there, it is built from the sources beside this file first; if that build
fails, importing this module fails: there is no fallback.
"""
from __future__ import annotations

import ctypes
import importlib.util
import os
import sys

import numpy as np
import torch  # noqa: F401  (plumbing: device memory and streams; loads the HIP runtime first)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libteuk.so")


def _build_missing_library() -> None:
    print(f"{LIB_PATH} not found: building it with hipcc (gfx950)", file=sys.stderr, flush=True)
    spec = importlib.util.spec_from_file_location("_teuk_build", os.path.join(_HERE, "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    try:
        mod.build(verbose=False)
    except Exception as e:  # noqa: BLE001
        raise ImportError(f"{LIB_PATH} is not built and building it failed: {e}") from e
    print(f"built {LIB_PATH}", file=sys.stderr, flush=True)


if not os.path.exists(LIB_PATH):
    _build_missing_library()

_lib = ctypes.CDLL(LIB_PATH)

TEUK_ABI_VERSION = 2
TEUK_OK = 0
TEUK_ERR_INVALID_ARG = -1
TEUK_ERR_OUT_OF_MEMORY = -2
TEUK_ERR_DEVICE = -3
TEUK_ERR_STATE = -4
TEUK_ERR_NONFINITE = -5
TEUK_ERR_UNSUPPORTED = -6
TEUK_ERR_CAPACITY = -7
TEUK_CHART_TORTOISE, TEUK_CHART_HYPERBOLOIDAL = 0, 1
TEUK_W_FP64, TEUK_W_FP32, TEUK_W_FP16, TEUK_W_BF16, TEUK_W_DD = 0, 1, 2, 3, 4
TEUK_S_FP64, TEUK_S_DD = 0, 1
TEUK_RK_SSP33, TEUK_RK_SSP104, TEUK_RK_SSP33_BLOCKED, TEUK_RK_SSP33_PIPELINED = 0, 1, 2, 3
INTEGRATOR = {"rk3": TEUK_RK_SSP33, "rk104": TEUK_RK_SSP104, "rk3_blocked": TEUK_RK_SSP33_BLOCKED,
              "rk3_pipelined": TEUK_RK_SSP33_PIPELINED}
TEUK_SCHEME_WENO5, TEUK_SCHEME_WENO3, TEUK_SCHEME_FD6KO8 = 0, 1, 2
SCHEME = {"weno5": TEUK_SCHEME_WENO5, "weno3": TEUK_SCHEME_WENO3, "fd6ko8": TEUK_SCHEME_FD6KO8}
TEUK_X_STATE, TEUK_X_WAVEFORM, TEUK_X_TIMES, TEUK_X_COEFFS, TEUK_X_RHS, TEUK_X_HORIZON = 0, 1, 2, 3, 4, 5
TEUK_NCOEF = 10
CHART = {"T": TEUK_CHART_TORTOISE, "H": TEUK_CHART_HYPERBOLOIDAL}
WEIGHT_PREC = {"fp64": TEUK_W_FP64, "fp32": TEUK_W_FP32, "fp16": TEUK_W_FP16, "bf16": TEUK_W_BF16, "dd": TEUK_W_DD}
STATE_PREC = {"fp64": TEUK_S_FP64, "dd": TEUK_S_DD}

_STATUS_NAMES = {0: "TEUK_OK", -1: "TEUK_ERR_INVALID_ARG", -2: "TEUK_ERR_OUT_OF_MEMORY", -3: "TEUK_ERR_DEVICE",
                 -4: "TEUK_ERR_STATE", -5: "TEUK_ERR_NONFINITE", -6: "TEUK_ERR_UNSUPPORTED",
                 -7: "TEUK_ERR_CAPACITY"}


class teuk_config(ctypes.Structure):
    _fields_ = [("abi_version", ctypes.c_int32), ("s", ctypes.c_int32), ("m", ctypes.c_int32),
                ("chart", ctypes.c_int32), ("nr", ctypes.c_int32), ("ntheta", ctypes.c_int32),
                ("weight_prec", ctypes.c_int32), ("extract_every", ctypes.c_int32),
                ("max_samples", ctypes.c_int32), ("workgroups", ctypes.c_int32),
                ("state_prec", ctypes.c_int32), ("integrator", ctypes.c_int32),
                ("scheme", ctypes.c_int32), ("theta_order", ctypes.c_int32),
                ("M", ctypes.c_double), ("a", ctypes.c_double), ("x_min", ctypes.c_double),
                ("x_max", ctypes.c_double), ("dt", ctypes.c_double), ("cfl", ctypes.c_double),
                ("weno_eps", ctypes.c_double), ("x_extract", ctypes.c_double), ("S", ctypes.c_double),
                ("ko_sigma", ctypes.c_double)]


class teuk_device_ctx(ctypes.Structure):
    _fields_ = [("stream", ctypes.c_void_p), ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t)]


class teuk_info_t(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("t", ctypes.c_double), ("steps", ctypes.c_int64),
                ("samples", ctypes.c_int64), ("j_extract", ctypes.c_int32), ("workgroups", ctypes.c_int32),
                ("dt_bound", ctypes.c_double)]


_P = ctypes.POINTER
_dp = _P(ctypes.c_double)
_lib.teuk_default_config.argtypes = [_P(teuk_config)]
_lib.teuk_default_config.restype = None
_lib.teuk_footprint_bytes.argtypes = [_P(teuk_config)]
_lib.teuk_footprint_bytes.restype = ctypes.c_size_t
_lib.teuk_create.argtypes = [_P(teuk_config), _P(teuk_device_ctx), _P(ctypes.c_void_p)]
_lib.teuk_create.restype = ctypes.c_int
_lib.teuk_set_initial.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32]
_lib.teuk_set_initial.restype = ctypes.c_int
_lib.teuk_step.argtypes = [ctypes.c_void_p, ctypes.c_int64]
_lib.teuk_step.restype = ctypes.c_int
_lib.teuk_extract.argtypes = [ctypes.c_void_p, ctypes.c_int32, _dp, ctypes.c_size_t, _P(ctypes.c_size_t)]
_lib.teuk_extract.restype = ctypes.c_int
_lib.teuk_info.argtypes = [ctypes.c_void_p, _P(teuk_info_t)]
_lib.teuk_info.restype = ctypes.c_int
_lib.teuk_check_finite.argtypes = [ctypes.c_void_p]
_lib.teuk_check_finite.restype = ctypes.c_int
_lib.teuk_destroy.argtypes = [ctypes.c_void_p]
_lib.teuk_destroy.restype = None
_lib.teuk_last_error.argtypes = [ctypes.c_void_p]
_lib.teuk_last_error.restype = ctypes.c_char_p
_lib.teuk_host_coefficients.argtypes = [_P(teuk_config), _dp, ctypes.c_size_t]
_lib.teuk_host_coefficients.restype = ctypes.c_int
class teuk_tune_info_t(ctypes.Structure):
    _fields_ = [("workgroups", ctypes.c_int32), ("segs", ctypes.c_int32), ("default_workgroups", ctypes.c_int32),
                ("default_segs", ctypes.c_int32), ("candidates", ctypes.c_int32), ("steps", ctypes.c_int32),
                ("us_per_step", ctypes.c_double), ("us_per_step_default", ctypes.c_double)]


class teuk_group_tune_info_t(ctypes.Structure):
    _fields_ = [("rows_per_tile", ctypes.c_int32), ("block_mib", ctypes.c_int32),
                ("default_rows_per_tile", ctypes.c_int32), ("default_block_mib", ctypes.c_int32),
                ("candidates", ctypes.c_int32), ("steps", ctypes.c_int32),
                ("us_per_step", ctypes.c_double), ("us_per_step_default", ctypes.c_double)]


_lib.teuk_tune.argtypes = [_P(teuk_config), ctypes.c_int32, _P(teuk_tune_info_t)]
_lib.teuk_tune.restype = ctypes.c_int
_lib.teuk_tune_forget.argtypes = []
_lib.teuk_tune_forget.restype = None
_lib.teuk_tune_last_error.argtypes = []
_lib.teuk_tune_last_error.restype = ctypes.c_char_p
_lib.teuk_set_graph.argtypes = [ctypes.c_void_p, ctypes.c_int32]
_lib.teuk_set_graph.restype = ctypes.c_int
_lib.teuk_step_noalloc.argtypes = [_P(teuk_config), ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
_lib.teuk_step_noalloc.restype = ctypes.c_int


class teuk_group_info_t(ctypes.Structure):
    _fields_ = [("members", ctypes.c_int32), ("classes", ctypes.c_int32), ("workgroups", ctypes.c_int64),
                ("tiles", ctypes.c_int64), ("units", ctypes.c_int64), ("points", ctypes.c_int64)]


_lib.teuk_group_create.argtypes = [_P(teuk_device_ctx), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                   _P(ctypes.c_void_p)]
_lib.teuk_group_create.restype = ctypes.c_int
_lib.teuk_group_add.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
_lib.teuk_group_add.restype = ctypes.c_int
_lib.teuk_group_remove.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
_lib.teuk_group_remove.restype = ctypes.c_int
_lib.teuk_group_step.argtypes = [ctypes.c_void_p, ctypes.c_int64]
_lib.teuk_group_step.restype = ctypes.c_int
_lib.teuk_group_tune.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]
_lib.teuk_group_tune.restype = ctypes.c_int
_lib.teuk_group_set_graph.argtypes = [ctypes.c_void_p, ctypes.c_int32]
_lib.teuk_group_set_graph.restype = ctypes.c_int
_lib.teuk_group_info.argtypes = [ctypes.c_void_p, _P(teuk_group_info_t)]
_lib.teuk_group_info.restype = ctypes.c_int
_lib.teuk_group_destroy.argtypes = [ctypes.c_void_p]
_lib.teuk_group_destroy.restype = None
_lib.teuk_group_last_error.argtypes = [ctypes.c_void_p]
_lib.teuk_group_last_error.restype = ctypes.c_char_p

EXPORTED = ["teuk_default_config", "teuk_footprint_bytes", "teuk_create", "teuk_set_initial", "teuk_step",
            "teuk_extract", "teuk_info", "teuk_check_finite", "teuk_destroy", "teuk_last_error",
            "teuk_host_coefficients", "teuk_group_create", "teuk_group_add", "teuk_group_remove",
            "teuk_group_step", "teuk_group_info", "teuk_group_destroy", "teuk_group_last_error",
            "teuk_step_noalloc", "teuk_set_graph", "teuk_group_set_graph", "teuk_tune", "teuk_tune_forget",
            "teuk_tune_last_error", "teuk_group_tune"]


class TeukError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def _check(st: int, h=None):
    if st != TEUK_OK:
        raise TeukError(st, _lib.teuk_last_error(h).decode())


def _gcheck(st: int, g=None):
    if st != TEUK_OK:
        raise TeukError(st, _lib.teuk_group_last_error(g).decode())


# ----------------------------------------------------------------------------- same names as the C ABI
def teuk_default_config() -> teuk_config:
    c = teuk_config()
    _lib.teuk_default_config(ctypes.byref(c))
    return c


def teuk_footprint_bytes(cfg: teuk_config) -> int:
    return int(_lib.teuk_footprint_bytes(ctypes.byref(cfg)))


def teuk_create(cfg: teuk_config, ctx: teuk_device_ctx | None = None) -> int:
    h = ctypes.c_void_p()
    st = _lib.teuk_create(ctypes.byref(cfg), ctypes.byref(ctx) if ctx is not None else None, ctypes.byref(h))
    _check(st)
    return h.value


def teuk_set_initial(h: int, u) -> None:
    if isinstance(u, torch.Tensor):
        if u.dtype != torch.float64 or not u.is_contiguous() or not u.is_cuda:
            raise ValueError("device initial data must be a contiguous float64 CUDA tensor")
        _check(_lib.teuk_set_initial(h, ctypes.c_void_p(u.data_ptr()), 1), h)
    else:
        a = np.ascontiguousarray(u, dtype=np.float64)
        _check(_lib.teuk_set_initial(h, a.ctypes.data_as(ctypes.c_void_p), 0), h)


def teuk_step(h: int, nsteps: int) -> None:
    _check(_lib.teuk_step(h, int(nsteps)), h)


def teuk_extract(h: int, what: int, capacity: int) -> np.ndarray:
    out = np.empty(max(int(capacity), 1), dtype=np.float64)
    written = ctypes.c_size_t(0)
    st = _lib.teuk_extract(h, int(what), out.ctypes.data_as(_dp), int(capacity), ctypes.byref(written))
    if st == TEUK_ERR_NONFINITE:
        raise TeukError(st, _lib.teuk_last_error(h).decode() + " (state copied for inspection)")
    _check(st, h)
    return out[: written.value]


def teuk_tune(cfg: teuk_config, steps: int = 0) -> teuk_tune_info_t:
    info = teuk_tune_info_t()
    st = _lib.teuk_tune(ctypes.byref(cfg), int(steps), ctypes.byref(info))
    if st != TEUK_OK:
        raise TeukError(st, _lib.teuk_tune_last_error().decode())
    return info


def teuk_tune_forget() -> None:
    _lib.teuk_tune_forget()


def teuk_tune_last_error() -> str:
    return _lib.teuk_tune_last_error().decode()


def teuk_set_graph(h: int, chunk_steps: int) -> None:
    _check(_lib.teuk_set_graph(h, int(chunk_steps)), h)


def teuk_info(h: int) -> teuk_info_t:
    info = teuk_info_t()
    _check(_lib.teuk_info(h, ctypes.byref(info)), h)
    return info


def teuk_check_finite(h: int) -> None:
    _check(_lib.teuk_check_finite(h), h)


def teuk_destroy(h: int | None) -> None:
    _lib.teuk_destroy(h)


def teuk_last_error(h: int | None = None) -> str:
    return _lib.teuk_last_error(h).decode()


def teuk_host_coefficients(cfg: teuk_config) -> np.ndarray:
    """[TEUK_NCOEF][ntheta][nr] (FP64 state) or [TEUK_NCOEF][ntheta][nr][2] pairs (double-double)."""
    n = cfg.nr * cfg.ntheta
    pv = 2 if cfg.state_prec == TEUK_S_DD else 1
    out = np.empty(TEUK_NCOEF * n * pv, dtype=np.float64)
    _check(_lib.teuk_host_coefficients(ctypes.byref(cfg), out.ctypes.data_as(_dp), out.size))
    return out.reshape((TEUK_NCOEF, cfg.ntheta, cfg.nr) + ((2,) if pv == 2 else ()))


def teuk_step_noalloc(cfg: teuk_config, u: "torch.Tensor", nsteps: int, stream=None) -> None:
    """Advance the contiguous float64 device tensor u ([4][ntheta][nr]) in place."""
    if not (isinstance(u, torch.Tensor) and u.is_cuda and u.dtype == torch.float64 and u.is_contiguous()):
        raise ValueError("u must be a contiguous float64 CUDA tensor")
    if u.numel() != 4 * cfg.nr * cfg.ntheta:
        raise ValueError(f"u holds {u.numel()} values, the grid needs {4 * cfg.nr * cfg.ntheta}")
    s = stream if stream is not None else torch.cuda.current_stream(u.device)
    _check(_lib.teuk_step_noalloc(ctypes.byref(cfg), ctypes.c_void_p(u.data_ptr()), int(nsteps),
                                  ctypes.c_void_p(s.cuda_stream)))


def teuk_group_create(ctx: teuk_device_ctx | None, max_members: int, workgroups: int = 0,
                      rows_per_tile: int = 0) -> int:
    g = ctypes.c_void_p()
    _gcheck(_lib.teuk_group_create(ctypes.byref(ctx) if ctx is not None else None, int(max_members),
                                   int(workgroups), int(rows_per_tile), ctypes.byref(g)))
    return g.value


def teuk_group_add(g: int, h: int) -> None:
    _gcheck(_lib.teuk_group_add(g, h), g)


def teuk_group_remove(g: int, h: int) -> None:
    _gcheck(_lib.teuk_group_remove(g, h), g)


def teuk_group_step(g: int, nsteps: int) -> None:
    _gcheck(_lib.teuk_group_step(g, int(nsteps)), g)


def teuk_group_tune(g: int, steps: int = 0) -> teuk_group_tune_info_t:
    info = teuk_group_tune_info_t()
    _gcheck(_lib.teuk_group_tune(g, int(steps), ctypes.byref(info)), g)
    return info


def teuk_group_set_graph(g: int, chunk_steps: int) -> None:
    _gcheck(_lib.teuk_group_set_graph(g, int(chunk_steps)), g)


def teuk_group_info(g: int) -> teuk_group_info_t:
    info = teuk_group_info_t()
    _gcheck(_lib.teuk_group_info(g, ctypes.byref(info)), g)
    return info


def teuk_group_destroy(g: int | None) -> None:
    _lib.teuk_group_destroy(g)


def teuk_group_last_error(g: int | None = None) -> str:
    return _lib.teuk_group_last_error(g).decode()


# ----------------------------------------------------------------------------- convenience (marshalling only)
def make_config(*, s: int, m: int, a: float, nr: int, ntheta: int, x_min: float, x_max: float,
                M: float = 1.0, dt: float = 0.0, cfl: float = 0.5, weno_eps: float = 1e-6,
                weight_prec="fp64", x_extract: float | None = None, extract_every: int = 0,
                max_samples: int = 0, workgroups: int = 0, chart="T", S: float = 20.0,
                state="fp64", integrator="rk3", scheme="weno5", ko_sigma: float = 0.01,
                theta_order: int = 2) -> teuk_config:
    c = teuk_default_config()
    c.s, c.m, c.a, c.M = int(s), int(m), float(a), float(M)
    c.nr, c.ntheta = int(nr), int(ntheta)
    c.x_min, c.x_max = float(x_min), float(x_max)
    c.dt, c.cfl, c.weno_eps = float(dt), float(cfl), float(weno_eps)
    c.weight_prec = WEIGHT_PREC[weight_prec] if isinstance(weight_prec, str) else int(weight_prec)
    c.extract_every, c.max_samples = int(extract_every), int(max_samples)
    c.x_extract = float(x_min if x_extract is None else x_extract)
    c.workgroups = int(workgroups)
    c.chart = CHART[chart] if isinstance(chart, str) else int(chart)
    c.S = float(S)
    c.state_prec = STATE_PREC[state] if isinstance(state, str) else int(state)
    c.integrator = INTEGRATOR[integrator] if isinstance(integrator, str) else int(integrator)
    c.scheme = SCHEME[scheme] if isinstance(scheme, str) else int(scheme)
    c.ko_sigma = float(ko_sigma)
    c.theta_order = int(theta_order)
    return c


class Solver:
    """One solve on the current CUDA (HIP) device.

    The solver's device buffers live in a torch uint8 workspace tensor held by
    this object, and its kernels run on `stream` (default: torch's current
    stream).  Methods map one-to-one onto the C ABI.
    """

    def __init__(self, cfg: teuk_config, stream: "torch.cuda.Stream | None" = None, device=None):
        self.cfg = cfg
        dev = torch.device("cuda") if device is None else torch.device(device)
        nbytes = teuk_footprint_bytes(cfg)
        if nbytes == 0:
            # let the library report why the configuration is invalid
            teuk_create(cfg, None)
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        base = self._ws.data_ptr()
        aligned = (base + 255) // 256 * 256
        self.ctx = teuk_device_ctx(ctypes.c_void_p(self.stream.cuda_stream), ctypes.c_void_p(aligned), nbytes)
        self.h = teuk_create(cfg, self.ctx)

    @property
    def dd(self) -> bool:
        """Double-double state: every value a (hi, lo) pair on a trailing axis."""
        return self.cfg.state_prec == TEUK_S_DD

    @property
    def plane_shape(self):
        return (4, self.cfg.ntheta, self.cfg.nr) + ((2,) if self.dd else ())

    def set_initial(self, u):
        """u: [4][ntheta][nr] (FP64 state); for the double-double state
        [4][ntheta][nr][2] pairs, or [4][ntheta][nr] doubles taken exactly (lo = 0)."""
        if self.dd and not isinstance(u, torch.Tensor):
            a = np.asarray(u, dtype=np.float64)
            if a.shape == (4, self.cfg.ntheta, self.cfg.nr):
                u = np.stack([a, np.zeros_like(a)], axis=-1)
        teuk_set_initial(self.h, u)

    def step(self, nsteps: int):
        teuk_step(self.h, nsteps)

    def set_graph(self, chunk_steps: int):
        """Graph mode: step() replays a captured graph of chunk_steps steps (0: off)."""
        teuk_set_graph(self.h, chunk_steps)

    def state(self) -> np.ndarray:
        n = int(np.prod(self.plane_shape))
        return teuk_extract(self.h, TEUK_X_STATE, n).reshape(self.plane_shape)

    def info(self) -> teuk_info_t:
        return teuk_info(self.h)

    def waveform(self):
        inf = self.info()
        ns = min(inf.samples, self.cfg.max_samples) if self.cfg.extract_every > 0 else 0
        pv = 2 if self.dd else 1
        w = teuk_extract(self.h, TEUK_X_WAVEFORM, ns * self.cfg.ntheta * 2 * pv)
        w = w.reshape((ns, self.cfg.ntheta, 2) + ((2,) if self.dd else ()))
        t = teuk_extract(self.h, TEUK_X_TIMES, ns)
        return t, w

    def horizon(self):
        """Horizon samples (hyperboloidal chart): times and complex arrays
        Phi_H[n][ntheta], dPhi_H[n][ntheta] (d_rho Phi) on rho_H."""
        inf = self.info()
        ns = min(inf.samples, self.cfg.max_samples) if self.cfg.extract_every > 0 else 0
        h = teuk_extract(self.h, TEUK_X_HORIZON, ns * self.cfg.ntheta * 4).reshape(ns, self.cfg.ntheta, 4)
        t = teuk_extract(self.h, TEUK_X_TIMES, ns)
        return t, h[..., 0] + 1j * h[..., 1], h[..., 2] + 1j * h[..., 3]

    def rhs(self) -> np.ndarray:
        """F(u^n) as the stage kernel evaluates it (the state is unchanged)."""
        n = int(np.prod(self.plane_shape))
        return teuk_extract(self.h, TEUK_X_RHS, n).reshape(self.plane_shape)

    def coefficients(self) -> np.ndarray:
        n = self.cfg.ntheta * self.cfg.nr * (2 if self.dd else 1)
        shape = (TEUK_NCOEF, self.cfg.ntheta, self.cfg.nr) + ((2,) if self.dd else ())
        return teuk_extract(self.h, TEUK_X_COEFFS, TEUK_NCOEF * n).reshape(shape)

    def check_finite(self):
        teuk_check_finite(self.h)

    def close(self):
        if self.h is not None:
            teuk_destroy(self.h)
            self.h = None
            self._ws = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Group:
    """Independent solves advanced together (one launch per RK stage for each
    cache block of members, a block running all of a step() call's steps
    before the next).  Members are ``Solver`` objects on the group's stream; the group
    keeps a reference to each so that their memory outlives membership."""

    def __init__(self, max_members: int, workgroups: int = 0, rows_per_tile: int = 0,
                 stream: "torch.cuda.Stream | None" = None, device=None):
        dev = torch.device("cuda") if device is None else torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        ctx = teuk_device_ctx(ctypes.c_void_p(self.stream.cuda_stream), None, 0)
        self.g = teuk_group_create(ctx, max_members, workgroups, rows_per_tile)
        self.members: list[Solver] = []

    def add(self, sv: "Solver"):
        teuk_group_add(self.g, sv.h)
        self.members.append(sv)

    def remove(self, sv: "Solver"):
        teuk_group_remove(self.g, sv.h)
        self.members.remove(sv)

    def step(self, nsteps: int):
        teuk_group_step(self.g, nsteps)

    def set_graph(self, chunk_steps: int):
        """Graph mode: each cache block replays a captured graph of chunk_steps steps (0: off)."""
        teuk_group_set_graph(self.g, chunk_steps)

    def tune(self, steps: int = 0) -> teuk_group_tune_info_t:
        """Time tile heights and cache-block sizes on clones of the members; apply the fastest."""
        return teuk_group_tune(self.g, steps)

    def info(self) -> teuk_group_info_t:
        return teuk_group_info(self.g)

    def close(self):
        if self.g is not None:
            teuk_group_destroy(self.g)
            self.g = None
            self.members = []

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
