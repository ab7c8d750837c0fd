"""Independent test-only references used to pin the oracle.

Nothing here shares code with ``oracle/`` or with the HIP library: these are
closed forms and a Fourier-space integrator of the semi-discrete Cahn-Hilliard
flow, written with numpy's FFT.
"""
from __future__ import annotations

import numpy as np

MASK64 = (1 << 64) - 1


def splitmix64_py(seed: int, k: int) -> int:
    """k-th output (k >= 1) of SplitMix64 seeded with `seed` (Steele, Lea and
    Flood, 2014): the state advances by 0x9e3779b97f4a7c15 per output and is
    passed through the variant-13 mixing function."""
    z = (seed + k * 0x9E3779B97F4A7C15) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def lam1(n: int, L: float) -> np.ndarray:
    """Eigenvalues of -D (periodic second difference, spacing L/n) on the FFT
    wavenumbers: (4/h^2) sin^2(k h / 2)."""
    h = L / n
    k = 2 * np.pi * np.fft.fftfreq(n, d=h)
    return (4.0 / h**2) * np.sin(k * h / 2) ** 2


def lam_grid(shape, L=2 * np.pi):
    """Eigenvalue of -lap_h for every Fourier mode of a (.., y, x) grid."""
    dim = len(shape)
    lam = np.zeros(shape)
    for ax in range(dim):
        s = [1] * dim
        s[ax] = shape[ax]
        lam = lam + lam1(shape[ax], L).reshape(s)
    return lam


def semi_discrete_flow(C0: np.ndarray, gamma: float, T: float, dt: float, L=2 * np.pi):
    """Integrate dC/dt = lap_h(C^3 - C - gamma lap_h C) (the spatially discrete
    Cahn-Hilliard system, no time splitting) with integrating-factor RK4 in
    Fourier space.  Its time error is O(dt^4), far below the O(dt) of the ADI
    scheme under test."""
    lam = lam_grid(C0.shape, L)
    lin = -gamma * lam**2
    fftn, ifftn = np.fft.fftn, np.fft.ifftn

    def nl(v):
        C = np.real(ifftn(v))
        return -lam * fftn(C**3 - C)

    v = fftn(C0)
    nst = int(round(T / dt))
    E = np.exp(lin * dt / 2)
    E2 = E * E
    for _ in range(nst):
        a = nl(v)
        b = nl(E * (v + dt / 2 * a))
        c = nl(E * v + dt / 2 * b)
        d = nl(E2 * v + dt * E * c)
        v = E2 * v + dt / 6 * (E2 * a + 2 * E * (b + c) + d)
    return np.real(ifftn(v))


def amplification(k, n, L, gamma, dt, c0, theta=1.0):
    """Closed-form growth factor of the linearised theta-weighted ADI step
    (theta = 1: implicit, 1/2: Crank-Nicolson) for the single Fourier mode
    cos(k.x) about the uniform state c0 (2D or 3D)."""
    lam = [(4.0 * n[d] ** 2 / L**2) * np.sin(np.pi * k[d] / n[d]) ** 2 for d in range(len(k))]
    num = 1.0
    for d in range(len(k)):
        num *= 1.0 - (1.0 - theta) * gamma * dt * lam[d] ** 2
    num -= dt * sum(lam) * (3 * c0**2 - 1)
    cross = sum(lam[d] * lam[e] for d in range(len(k)) for e in range(d + 1, len(k)))
    num -= 2 * gamma * dt * cross
    den = 1.0
    for d in range(len(k)):
        den *= 1.0 + theta * gamma * dt * lam[d] ** 2
    return num / den
