"""Thin ctypes binding of libch.so (the C ABI declared in include/ch.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of libch.so.  PyTorch provides the device workspace and the stream.
The functions keep the C names; ``Ensemble`` bundles a context with its
workspace tensor.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libch.so")

CH_OK, CH_EINVAL, CH_ENOMEM, CH_EDEVICE, CH_ESTATE, CH_ENONFINITE, CH_EUNSUPPORTED = range(7)
CH_F64, CH_F32_BULK = 0, 1
CH_ENERGY_QUARTER, CH_ENERGY_PAPER_PRINTED = 0, 1

STATUS_NAMES = {
    CH_OK: "CH_OK", CH_EINVAL: "CH_EINVAL", CH_ENOMEM: "CH_ENOMEM", CH_EDEVICE: "CH_EDEVICE",
    CH_ESTATE: "CH_ESTATE", CH_ENONFINITE: "CH_ENONFINITE", CH_EUNSUPPORTED: "CH_EUNSUPPORTED",
}

EXPORTED = (
    "ch_workspace_bytes", "ch_create", "ch_init_random", "ch_set_field", "ch_get_field",
    "ch_get_step", "ch_set_step", "ch_step", "ch_energy", "ch_beta_series", "ch_autotune",
    "ch_set_graph_steps", "ch_describe", "ch_time_kernels", "ch_destroy", "ch_last_error",
    "ch_version", "ch_solver_coefficients", "ch_num_classes", "ch_set_tiles",
    "ch_ensemble_moments", "ch_ensemble_window", "ch_beta_histogram", "ch_sync_step",
    "ch_step_static", "ch_set_theta",
)

# Allocation-free stepping (ch_step_static): limits of its static device scratch
CH_STATIC_SCRATCH_BYTES = 80 << 20
CH_STATIC_MAX_MEMBERS = 64


class ChError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class ch_member_desc(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32),
        ("n", ctypes.c_int32 * 3),
        ("L", ctypes.c_double * 3),
        ("gamma", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("c0", ctypes.c_double),
        ("noise", ctypes.c_double),
        ("seed", ctypes.c_uint64),
    ]


_lib = None


def load() -> ctypes.CDLL:
    """Load libch.so; raise if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`"
            " (there is no CPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    dp, vp, i64p = P(ctypes.c_double), ctypes.c_void_p, P(ctypes.c_int64)
    sig = {
        "ch_workspace_bytes": (ctypes.c_size_t, [P(ch_member_desc), ctypes.c_int32, ctypes.c_int,
                                                 ctypes.c_int32, ctypes.c_int64]),
        "ch_create": (ctypes.c_int, [P(ch_member_desc), ctypes.c_int32, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_int32, ctypes.c_int64, vp, ctypes.c_size_t, vp,
                                     P(vp)]),
        "ch_init_random": (ctypes.c_int, [vp]),
        "ch_set_field": (ctypes.c_int, [vp, ctypes.c_int32, dp]),
        "ch_get_field": (ctypes.c_int, [vp, ctypes.c_int32, dp]),
        "ch_get_step": (ctypes.c_int, [vp, i64p]),
        "ch_set_step": (ctypes.c_int, [vp, ctypes.c_int64]),
        "ch_step": (ctypes.c_int, [vp, ctypes.c_int64]),
        "ch_energy": (ctypes.c_int, [vp, dp, dp]),
        "ch_beta_series": (ctypes.c_int, [vp, ctypes.c_int32, dp, dp, dp, dp, dp, dp, ctypes.c_int64,
                                          i64p]),
        "ch_autotune": (ctypes.c_int, [vp, ctypes.c_char_p]),
        "ch_set_graph_steps": (ctypes.c_int, [vp, ctypes.c_int32]),
        "ch_describe": (ctypes.c_int, [vp, ctypes.c_char_p, ctypes.c_size_t]),
        "ch_time_kernels": (ctypes.c_int, [vp, ctypes.c_int64, dp]),
        "ch_destroy": (ctypes.c_int, [vp]),
        "ch_last_error": (ctypes.c_char_p, [vp]),
        "ch_version": (ctypes.c_char_p, []),
        "ch_solver_coefficients": (ctypes.c_int, [ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                                  ctypes.c_int32, dp]),
        "ch_num_classes": (ctypes.c_int, [vp, P(ctypes.c_int32)]),
        "ch_set_tiles": (ctypes.c_int, [vp] + [ctypes.c_int32] * 9),
        "ch_sync_step": (ctypes.c_int, [vp, i64p]),
        "ch_set_theta": (ctypes.c_int, [vp, ctypes.c_double]),
        "ch_step_static": (ctypes.c_int, [P(ch_member_desc), ctypes.c_int32, ctypes.c_int, vp,
                                          ctypes.c_int64, vp, vp]),
        "ch_ensemble_moments": (ctypes.c_int, [vp, P(ctypes.c_int32), ctypes.c_int32, ctypes.c_int32, dp,
                                               dp, ctypes.c_int64, i64p]),
        "ch_ensemble_window": (ctypes.c_int, [vp, P(ctypes.c_int32), ctypes.c_int32, ctypes.c_double,
                                              ctypes.c_double, dp, dp]),
        "ch_beta_histogram": (ctypes.c_int, [vp, P(ctypes.c_int32), ctypes.c_int32, ctypes.c_double,
                                             ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                             ctypes.c_int32, P(ctypes.c_uint64)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _dp(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def last_error(ctx=None) -> str:
    msg = load().ch_last_error(ctx)
    return msg.decode() if msg else ""


def _check(status: int, ctx=None):
    if status != CH_OK:
        raise ChError(status, last_error(ctx))


def make_desc(n: Sequence[int], gamma: float, dt: float, c0: float = 0.0, noise: float = 0.0,
              seed: int = 0, L: Optional[Sequence[float]] = None) -> ch_member_desc:
    """Descriptor of one member; n is (nx, ny) or (nx, ny, nz), x fastest."""
    dim = len(n)
    d = ch_member_desc()
    d.dim = dim
    nn = list(n) + [1] * (3 - dim)
    d.n = (ctypes.c_int32 * 3)(*nn)
    if L is None:
        L = [2 * np.pi] * dim
    LL = list(L) + [1.0] * (3 - dim)
    d.L = (ctypes.c_double * 3)(*LL)
    d.gamma, d.dt, d.c0, d.noise, d.seed = gamma, dt, c0, noise, seed
    return d


def desc_array(descs: Sequence[ch_member_desc]):
    arr = (ch_member_desc * len(descs))()
    for i, d in enumerate(descs):
        arr[i] = d
    return arr


def ch_workspace_bytes(descs, prec=CH_F64, cadence=10, max_samples=1) -> int:
    arr = desc_array(descs)
    nb = load().ch_workspace_bytes(arr, len(descs), prec, cadence, max_samples)
    if nb == 0:
        raise ChError(CH_EINVAL, last_error())
    return nb


def ch_solver_coefficients(rho: float, n: int, chunk: int, prec: int = CH_F64) -> np.ndarray:
    out = np.zeros(11, dtype=np.float64)
    _check(load().ch_solver_coefficients(rho, n, chunk, prec, _dp(out)))
    return out


def ch_step_static(descs, prec, field, nsteps: int, energy=None, stream=None):
    """Advance the device tensor `field` (members back to back, each x-fastest,
    float64 for CH_F64 or float32 for CH_F32_BULK) in place by nsteps steps
    without any device allocation; `energy` (optional float64 device tensor of
    4 * len(descs) values) receives F, <C>, G_id and nsteps per member.
    Enqueued on `stream` (a torch stream; None = torch's current stream)."""
    import torch

    arr = desc_array(descs)
    if stream is None:
        stream = torch.cuda.current_stream()
    st = load().ch_step_static(arr, len(descs), prec, ctypes.c_void_p(field.data_ptr()), nsteps,
                               ctypes.c_void_p(energy.data_ptr()) if energy is not None else None,
                               ctypes.c_void_p(stream.cuda_stream))
    _check(st)


@dataclass
class Ensemble:
    """A context plus the caller-owned workspace it lives in."""
    descs: list
    prec: int = CH_F64
    conv: int = CH_ENERGY_QUARTER
    cadence: int = 10
    max_samples: int = 1
    stream: object = None
    ctx: ctypes.c_void_p = field(default=None, init=False)
    ws: object = field(default=None, init=False)

    def __post_init__(self):
        import torch

        lib = load()
        arr = desc_array(self.descs)
        nbytes = ch_workspace_bytes(self.descs, self.prec, self.cadence, self.max_samples)
        # torch allocations are at least 256-byte aligned
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        if self.stream is None:
            # a stream of our own (default priority): the legacy null stream
            # cannot be captured into HIP graphs
            self.stream = torch.cuda.Stream()
        ctx = ctypes.c_void_p()
        st = lib.ch_create(arr, len(self.descs), self.prec, self.conv, self.cadence,
                           self.max_samples, ctypes.c_void_p(self.ws.data_ptr()), nbytes,
                           ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(ctx))
        _check(st)
        self.ctx = ctx

    # -- state --------------------------------------------------------------
    @property
    def m(self) -> int:
        return len(self.descs)

    def shape(self, member: int):
        d = self.descs[member]
        return tuple(d.n[a] for a in range(d.dim))[::-1]  # numpy order (z, y, x)

    def init_random(self):
        _check(load().ch_init_random(self.ctx), self.ctx)

    def set_field(self, member: int, C: np.ndarray):
        C = np.ascontiguousarray(C, dtype=np.float64)
        assert C.shape == self.shape(member)
        _check(load().ch_set_field(self.ctx, member, _dp(C)), self.ctx)

    def get_field(self, member: int) -> np.ndarray:
        out = np.empty(self.shape(member), dtype=np.float64)
        _check(load().ch_get_field(self.ctx, member, _dp(out)), self.ctx)
        return out

    @property
    def step_count(self) -> int:
        n = ctypes.c_int64()
        _check(load().ch_get_step(self.ctx, ctypes.byref(n)), self.ctx)
        return n.value

    def set_step(self, n: int):
        _check(load().ch_set_step(self.ctx, n), self.ctx)

    def sync_step(self) -> int:
        """Read the device step counter back (after replays of a graph the
        caller captured) and return it."""
        n = ctypes.c_int64()
        _check(load().ch_sync_step(self.ctx, ctypes.byref(n)), self.ctx)
        return n.value

    def step(self, nsteps: int):
        _check(load().ch_step(self.ctx, nsteps), self.ctx)

    def energy(self):
        F = np.empty(self.m)
        mC = np.empty(self.m)
        _check(load().ch_energy(self.ctx, _dp(F), _dp(mC)), self.ctx)
        return F, mC

    def beta_series(self, member: int) -> np.ndarray:
        """(J, 6) array: t, F, dF/dt (time difference), dF/dt (identity), beta, <C>."""
        cap = self.max_samples
        cols = [np.empty(cap) for _ in range(6)]
        count = ctypes.c_int64()
        _check(load().ch_beta_series(self.ctx, member, *[_dp(c) for c in cols], cap,
                                     ctypes.byref(count)), self.ctx)
        J = count.value
        return np.stack([c[:J] for c in cols], axis=1)

    def _members(self, members):
        if members is None:
            return None, 0
        sel = np.ascontiguousarray(members, dtype=np.int32)
        return sel, len(sel)

    def ensemble_moments(self, members=None, pmax: int = 4):
        """(t, mu): t (J,), mu (J, pmax) with mu[:, 0] the ensemble mean of beta
        and mu[:, p-1] its p-th central moment, over `members` (default all)."""
        sel, nm = self._members(members)
        cap = self.max_samples
        t = np.empty(cap)
        mu = np.empty(cap * pmax)
        count = ctypes.c_int64()
        mp = sel.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) if sel is not None else None
        _check(load().ch_ensemble_moments(self.ctx, mp, nm, pmax, _dp(t), _dp(mu), cap,
                                          ctypes.byref(count)), self.ctx)
        J = count.value
        return t[:J], mu[:J * pmax].reshape(J, pmax)

    def ensemble_window(self, t1: float, t2: float, members=None):
        """(beta0, k): time average of the ensemble-mean beta over [t1, t2] and the
        least-squares slope of its variance, mu_2 = k t."""
        sel, nm = self._members(members)
        b0, k = ctypes.c_double(), ctypes.c_double()
        mp = sel.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) if sel is not None else None
        _check(load().ch_ensemble_window(self.ctx, mp, nm, t1, t2, ctypes.byref(b0), ctypes.byref(k)),
               self.ctx)
        return b0.value, k.value

    def beta_histogram(self, t1: float, t2: float, lo: float, hi: float, nbins: int, members=None):
        """Counts of beta over the members and samples with t in [t1, t2]:
        [below lo, nbins bins of [lo, hi), at or above hi]."""
        sel, nm = self._members(members)
        counts = np.zeros(nbins + 2, dtype=np.uint64)
        mp = sel.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) if sel is not None else None
        _check(load().ch_beta_histogram(self.ctx, mp, nm, t1, t2, lo, hi, nbins,
                                        counts.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))), self.ctx)
        return counts

    def autotune(self, cache_path: Optional[str] = None):
        _check(load().ch_autotune(self.ctx, cache_path.encode() if cache_path else None), self.ctx)

    def num_classes(self) -> int:
        n = ctypes.c_int32()
        _check(load().ch_num_classes(self.ctx, ctypes.byref(n)), self.ctx)
        return n.value

    def set_tiles(self, cls: int, cx: int, rl: int, waves: int, units: int, cy: int, by: int,
                  cz: int = 0, bz: int = 0):
        _check(load().ch_set_tiles(self.ctx, cls, cx, rl, waves, units, cy, by, cz, bz), self.ctx)

    def set_theta(self, theta: float):
        """Time scheme: 1 = implicit ADI (default), 0.5 = Crank-Nicolson ADI (2D)."""
        _check(load().ch_set_theta(self.ctx, theta), self.ctx)

    def set_graph_steps(self, g: int):
        _check(load().ch_set_graph_steps(self.ctx, g), self.ctx)

    def describe(self) -> str:
        buf = ctypes.create_string_buffer(8192)
        _check(load().ch_describe(self.ctx, buf, len(buf)), self.ctx)
        return buf.value.decode()

    def time_kernels(self, nsteps: int) -> np.ndarray:
        ms = np.zeros(3)
        _check(load().ch_time_kernels(self.ctx, nsteps, _dp(ms)), self.ctx)
        return ms

    def close(self):
        if self.ctx:
            _check(load().ch_destroy(self.ctx))
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
