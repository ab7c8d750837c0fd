"""FP64 CPU oracle for the Cahn-Hilliard ensemble hot path.

TEST INFRASTRUCTURE ONLY: this package is the parity reference for the HIP
library.  Only the tests, the smoke check and the CPU-baseline leg of the
benchmark import it; the product path never does, and it shares no code with
the HIP path.

The arithmetic lives in ``ch_oracle.c`` (plain loops, FP64, exactly rounded
sums); this module only loads it with ctypes and marshals numpy arrays.

Paper references: the PDE is eq. (ch) of Section 1, the free energy and its
rate are eq. (dFdt_ch), the coarsening rate is eq. (betadef); the method is the
semi-implicit ADI finite-difference scheme of Section 4.1 / Appendix A.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ch_oracle.c")
_LIB = os.path.join(_HERE, "libch_oracle.so")

ENERGY_QUARTER = 0
ENERGY_PAPER_PRINTED = 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP).  Returns the library path."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-std=c99", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        L.orc_splitmix64.restype = ctypes.c_uint64
        L.orc_splitmix64.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.orc_uniform.restype = ctypes.c_double
        L.orc_uniform.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.orc_init_field.restype = None
        L.orc_init_field.argtypes = [ctypes.c_int, ip, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_uint64, dp]
        L.orc_exact_sum.restype = ctypes.c_double
        L.orc_exact_sum.argtypes = [dp, ctypes.c_int64]
        for name in ("orc_laplacian", "orc_cross"):
            f = getattr(L, name)
            f.restype = None
            f.argtypes = [ctypes.c_int, ip, dp, dp, dp]
        L.orc_cyclic_penta_solve.restype = ctypes.c_int
        L.orc_cyclic_penta_solve.argtypes = [ctypes.c_int64, ctypes.c_double, dp, dp]
        L.orc_rhs.restype = None
        L.orc_rhs.argtypes = [ctypes.c_int, ip, dp, ctypes.c_double, ctypes.c_double, dp, dp]
        L.orc_step.restype = ctypes.c_int
        L.orc_step.argtypes = [ctypes.c_int, ip, dp, ctypes.c_double, ctypes.c_double, dp,
                               ctypes.c_int64]
        L.orc_step_theta.restype = ctypes.c_int
        L.orc_step_theta.argtypes = [ctypes.c_int, ip, dp, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, dp, ctypes.c_int64]
        L.orc_energy.restype = ctypes.c_double
        L.orc_energy.argtypes = [ctypes.c_int, ip, dp, ctypes.c_double, ctypes.c_int, dp]
        L.orc_mean.restype = ctypes.c_double
        L.orc_mean.argtypes = [ctypes.c_int, ip, dp]
        L.orc_dFdt_identity.restype = ctypes.c_double
        L.orc_dFdt_identity.argtypes = [ctypes.c_int, ip, dp, ctypes.c_double, dp]
        L.orc_run_series.restype = ctypes.c_int64
        L.orc_run_series.argtypes = [ctypes.c_int, ip, dp, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_int, ctypes.c_int32, ctypes.c_int64, dp, dp,
                                     ctypes.c_int64]
        L.orc_run_series_theta.restype = ctypes.c_int64
        L.orc_run_series_theta.argtypes = [ctypes.c_int, ip, dp, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_double, ctypes.c_int, ctypes.c_int32, ctypes.c_int64,
                                           dp, dp, ctypes.c_int64]
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_num_threads.argtypes = []
        L.orc_set_num_threads.restype = ctypes.c_int
        L.orc_set_num_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _dims(shape):
    """numpy shape (z, y, x) or (y, x) -> (dim, int32[3] with x fastest)."""
    dim = len(shape)
    n = np.ones(3, dtype=np.int32)
    for d in range(dim):
        n[d] = shape[dim - 1 - d]
    return dim, n


def _lengths(dim, L):
    if np.isscalar(L):
        L = [L] * dim
    arr = np.ones(3, dtype=np.float64)
    arr[:dim] = L
    return arr


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def splitmix64(seed: int, k: int) -> int:
    return lib().orc_splitmix64(seed, k)


def uniform(seed: int, site: int) -> float:
    return lib().orc_uniform(seed, site)


def init_field(shape, c0: float, noise: float, seed: int) -> np.ndarray:
    dim, n = _dims(shape)
    C = np.empty(shape, dtype=np.float64)
    lib().orc_init_field(dim, _ip(n), c0, noise, seed, _dp(C))
    return C


def exact_sum(x) -> float:
    x = np.ascontiguousarray(x, dtype=np.float64).ravel()
    return lib().orc_exact_sum(_dp(x), x.size)


def laplacian(f: np.ndarray, L=2 * np.pi) -> np.ndarray:
    f = np.ascontiguousarray(f, dtype=np.float64)
    dim, n = _dims(f.shape)
    out = np.empty_like(f)
    lib().orc_laplacian(dim, _ip(n), _dp(_lengths(dim, L)), _dp(f), _dp(out))
    return out


def cross(f: np.ndarray, L=2 * np.pi) -> np.ndarray:
    f = np.ascontiguousarray(f, dtype=np.float64)
    dim, n = _dims(f.shape)
    out = np.empty_like(f)
    lib().orc_cross(dim, _ip(n), _dp(_lengths(dim, L)), _dp(f), _dp(out))
    return out


def cyclic_penta_solve(rho: float, f) -> np.ndarray:
    f = np.ascontiguousarray(f, dtype=np.float64)
    y = np.empty_like(f)
    rc = lib().orc_cyclic_penta_solve(f.size, rho, _dp(f), _dp(y))
    if rc != 0:
        raise ValueError(f"orc_cyclic_penta_solve failed ({rc})")
    return y


def rhs(C: np.ndarray, gamma: float, dt: float, L=2 * np.pi) -> np.ndarray:
    C = np.ascontiguousarray(C, dtype=np.float64)
    dim, n = _dims(C.shape)
    out = np.empty_like(C)
    lib().orc_rhs(dim, _ip(n), _dp(_lengths(dim, L)), gamma, dt, _dp(C), _dp(out))
    return out


def step(C: np.ndarray, gamma: float, dt: float, nsteps: int = 1, L=2 * np.pi,
         theta: float = 1.0) -> np.ndarray:
    """Return C advanced by nsteps ADI steps (input left untouched); theta = 1
    is the implicit ADI scheme, theta = 1/2 its Crank-Nicolson variant."""
    C = np.array(C, dtype=np.float64, order="C", copy=True)
    dim, n = _dims(C.shape)
    rc = lib().orc_step_theta(dim, _ip(n), _dp(_lengths(dim, L)), gamma, dt, theta, _dp(C), nsteps)
    if rc != 0:
        raise RuntimeError(f"orc_step failed ({rc})")
    return C


def energy(C: np.ndarray, gamma: float, L=2 * np.pi, conv: int = ENERGY_QUARTER) -> float:
    C = np.ascontiguousarray(C, dtype=np.float64)
    dim, n = _dims(C.shape)
    return lib().orc_energy(dim, _ip(n), _dp(_lengths(dim, L)), gamma, conv, _dp(C))


def mean(C: np.ndarray) -> float:
    C = np.ascontiguousarray(C, dtype=np.float64)
    dim, n = _dims(C.shape)
    return lib().orc_mean(dim, _ip(n), _dp(C))


def dFdt_identity(C: np.ndarray, gamma: float, L=2 * np.pi) -> float:
    C = np.ascontiguousarray(C, dtype=np.float64)
    dim, n = _dims(C.shape)
    return lib().orc_dFdt_identity(dim, _ip(n), _dp(_lengths(dim, L)), gamma, _dp(C))


SERIES_COLUMNS = ("t", "F", "dFdt", "dFdt_identity", "beta", "meanC")


def run_series(C: np.ndarray, gamma: float, dt: float, nsteps: int, K: int = 10,
               L=2 * np.pi, conv: int = ENERGY_QUARTER, theta: float = 1.0):
    """Run nsteps from C; return (final C, samples[J, 6]) with SERIES_COLUMNS."""
    C = np.array(C, dtype=np.float64, order="C", copy=True)
    dim, n = _dims(C.shape)
    J = nsteps // K + 1
    out = np.full((J, 6), np.nan, dtype=np.float64)
    got = lib().orc_run_series_theta(dim, _ip(n), _dp(_lengths(dim, L)), gamma, dt, theta, conv, K,
                                     nsteps, _dp(C), _dp(out), J)
    if got != J:
        raise RuntimeError(f"orc_run_series failed ({got})")
    return C, out


def num_threads() -> int:
    return lib().orc_num_threads()


def set_num_threads(n: int) -> int:
    """Use n OpenMP threads from now on; returns the previous count."""
    return lib().orc_set_num_threads(n)
