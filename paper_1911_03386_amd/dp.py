"""Thin ctypes binding of the droplet-population calls of libch.so (the C ABI
declared in include/dp.h): Model 1 ensembles.

Argument marshalling only: every step of the integration runs in the HIP
kernels of libch.so.  PyTorch provides the device workspace and the stream.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np

from .ch import CH_EINVAL, CH_ESTATE, CH_OK, STATUS_NAMES, load  # noqa: F401  (status codes re-exported)

EXPORTED = (
    "dp_workspace_bytes", "dp_create", "dp_set_radii", "dp_advance", "dp_run", "dp_member_info",
    "dp_get_volumes", "dp_series", "dp_ensemble_moments", "dp_ensemble_window", "dp_beta_histogram",
    "dp_destroy", "dp_last_error",
)

DP_RUNNING, DP_DONE, DP_UNDERFLOW, DP_NONFINITE, DP_ATTEMPT_LIMIT = range(5)
DP_MAX_DROPLETS = 8192
SLOTS = ("t", "F", "dFdt", "beta", "ubar", "alive")


class DpError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class dp_params(ctypes.Structure):
    _fields_ = [
        ("t_end", ctypes.c_double),
        ("dt_sample", ctypes.c_double),
        ("rtol", ctypes.c_double),
        ("atol", ctypes.c_double),
        ("h0", ctypes.c_double),
        ("max_attempts", ctypes.c_int64),
    ]


_bound = False


def lib() -> ctypes.CDLL:
    """libch.so with the dp_* signatures declared (raises if it is not built)."""
    global _bound
    L = load()
    if _bound:
        return L
    P = ctypes.POINTER
    vp, dp_, i32p, i64p = ctypes.c_void_p, P(ctypes.c_double), P(ctypes.c_int32), P(ctypes.c_int64)
    sig = {
        "dp_workspace_bytes": (ctypes.c_size_t, [i32p, ctypes.c_int32, P(dp_params)]),
        "dp_create": (ctypes.c_int, [i32p, ctypes.c_int32, P(dp_params), vp, ctypes.c_size_t, vp, P(vp)]),
        "dp_set_radii": (ctypes.c_int, [vp, dp_]),
        "dp_advance": (ctypes.c_int, [vp, ctypes.c_int64]),
        "dp_run": (ctypes.c_int, [vp, ctypes.c_int64, i64p, dp_]),
        "dp_member_info": (ctypes.c_int, [vp, ctypes.c_int32, dp_, i64p, i64p, i32p, i64p, dp_]),
        "dp_get_volumes": (ctypes.c_int, [vp, ctypes.c_int32, dp_]),
        "dp_series": (ctypes.c_int, [vp, ctypes.c_int32, dp_, ctypes.c_int64, i64p]),
        "dp_ensemble_moments": (ctypes.c_int, [vp, i32p, ctypes.c_int32, ctypes.c_int32, dp_, dp_,
                                               ctypes.c_int64, i64p]),
        "dp_ensemble_window": (ctypes.c_int, [vp, i32p, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                              dp_, dp_]),
        "dp_beta_histogram": (ctypes.c_int, [vp, i32p, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                             ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                             P(ctypes.c_uint64)]),
        "dp_destroy": (ctypes.c_int, [vp]),
        "dp_last_error": (ctypes.c_char_p, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _bound = True
    return L


def last_error(ctx=None) -> str:
    msg = lib().dp_last_error(ctx)
    return msg.decode() if msg else ""


def _check(status: int, ctx=None):
    if status != CH_OK:
        raise DpError(status, last_error(ctx))


def _i32(a: Sequence[int]):
    arr = np.ascontiguousarray(a, dtype=np.int32)
    return arr, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _f64p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_params(t_end: float, dt_sample: float = 0.1, rtol: float = 1e-6, atol: float = 1e-9, h0: float = 1e-4,
                max_attempts: int = 10**7) -> dp_params:
    return dp_params(t_end, dt_sample, rtol, atol, h0, max_attempts)


def workspace_bytes(n: Sequence[int], prm: dp_params) -> int:
    arr, p = _i32(n)
    nb = lib().dp_workspace_bytes(p, len(arr), ctypes.byref(prm))
    if nb == 0:
        # the same checks as dp_create, which reports the reason
        st = lib().dp_create(p, len(arr), ctypes.byref(prm), None, 0, None, ctypes.byref(ctypes.c_void_p()))
        _check(st)
    return nb


class DropletEnsemble:
    """A context over M droplet populations of sizes n[0..M-1], with the
    caller-owned workspace it lives in."""

    def __init__(self, n: Sequence[int], t_end: float, dt_sample: float = 0.1, rtol: float = 1e-6,
                 atol: float = 1e-9, h0: float = 1e-4, max_attempts: int = 10**7, stream=None):
        import torch

        self.n = [int(v) for v in n]
        self.prm = make_params(t_end, dt_sample, rtol, atol, h0, max_attempts)
        nbytes = workspace_bytes(self.n, self.prm)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self.stream = stream if stream is not None else torch.cuda.Stream()
        arr, p = _i32(self.n)
        ctx = ctypes.c_void_p()
        _check(lib().dp_create(p, len(arr), ctypes.byref(self.prm), ctypes.c_void_p(self.ws.data_ptr()), nbytes,
                               ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(ctx)))
        self.ctx = ctx
        self.J = int(round(t_end / dt_sample)) + 1

    @property
    def m(self) -> int:
        return len(self.n)

    def set_radii(self, radii: Sequence[np.ndarray]):
        """Initial radii per member (sample 0 is recorded, t = 0)."""
        flat = np.ascontiguousarray(np.concatenate([np.asarray(r, dtype=np.float64) for r in radii]))
        assert flat.size == sum(self.n)
        _check(lib().dp_set_radii(self.ctx, _f64p(flat)), self.ctx)

    def advance(self, attempts: int):
        _check(lib().dp_advance(self.ctx, attempts), self.ctx)

    def run(self, attempts: int = 4096):
        """Integrate every member to t_end; returns (launches, summed kernel ms)."""
        nl = ctypes.c_int64()
        ms = ctypes.c_double()
        _check(lib().dp_run(self.ctx, attempts, ctypes.byref(nl), ctypes.byref(ms)), self.ctx)
        return nl.value, ms.value

    def info(self, member: int) -> dict:
        t, evals = ctypes.c_double(), ctypes.c_double()
        acc, rej, samples = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        state = ctypes.c_int32()
        _check(lib().dp_member_info(self.ctx, member, ctypes.byref(t), ctypes.byref(acc), ctypes.byref(rej),
                                    ctypes.byref(state), ctypes.byref(samples), ctypes.byref(evals)), self.ctx)
        return dict(t=t.value, accepted=acc.value, rejected=rej.value, state=state.value, samples=samples.value,
                    evals=evals.value)

    def volumes(self, member: int) -> np.ndarray:
        out = np.empty(self.n[member])
        _check(lib().dp_get_volumes(self.ctx, member, _f64p(out)), self.ctx)
        return out

    def series(self, member: int) -> np.ndarray:
        """(count, 6): t, F, dF/dt, beta, ubar, live droplets."""
        out = np.empty((self.J, 6))
        cnt = ctypes.c_int64()
        _check(lib().dp_series(self.ctx, member, _f64p(out), self.J, ctypes.byref(cnt)), self.ctx)
        return out[:cnt.value].copy()

    def _members(self, members):
        if members is None:
            return None, None, self.m
        arr, p = _i32(members)
        return arr, p, len(arr)

    def ensemble_moments(self, members=None, pmax: int = 4):
        keep, p, nm = self._members(members)
        t = np.empty(self.J)
        mu = np.empty((self.J, pmax))
        cnt = ctypes.c_int64()
        _check(lib().dp_ensemble_moments(self.ctx, p, nm, pmax, _f64p(t), _f64p(mu), self.J, ctypes.byref(cnt)),
               self.ctx)
        return t[:cnt.value].copy(), mu[:cnt.value].copy()

    def ensemble_window(self, t1: float, t2: float, members=None):
        keep, p, nm = self._members(members)
        b0, k = ctypes.c_double(), ctypes.c_double()
        _check(lib().dp_ensemble_window(self.ctx, p, nm, t1, t2, ctypes.byref(b0), ctypes.byref(k)), self.ctx)
        return b0.value, k.value

    def beta_histogram(self, t1: float, t2: float, lo: float, hi: float, nbins: int, members=None):
        keep, p, nm = self._members(members)
        counts = np.zeros(nbins + 2, dtype=np.uint64)
        _check(lib().dp_beta_histogram(self.ctx, p, nm, t1, t2, lo, hi, nbins,
                                       counts.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))), self.ctx)
        return counts.astype(np.int64)

    def close(self):
        if getattr(self, "ctx", None):
            _check(lib().dp_destroy(self.ctx))
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
