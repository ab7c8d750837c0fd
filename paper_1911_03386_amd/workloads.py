"""Seeded synthetic workloads (ensemble recipes) shared by the benchmark and
the tests.  Only member descriptors are produced here: no part of the scheme.

The paper's ensembles (Section 4, Table "ensemblesCH") are M = 1024 periodic
2D realisations at gamma = 0.01 with i.i.d. uniform initial noise; these
recipes keep that structure at sizes one GPU finishes in seconds to minutes.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List

import numpy as np

from .ch import CH_F32_BULK, CH_F64, make_desc  # noqa: F401  (make_desc re-exported)

TWO_PI = 2 * np.pi


@dataclass
class Workload:
    name: str
    descs: list
    prec: int
    steps: int
    cadence: int = 10
    note: str = ""

    @property
    def sites(self) -> int:
        tot = 0
        for d in self.descs:
            s = 1
            for a in range(d.dim):
                s *= d.n[a]
            tot += s
        return tot


def c1() -> Workload:
    d = make_desc((128, 128), 0.01, 1e-3, c0=0.0, noise=0.1, seed=1)
    return Workload("ch2d_128x128_fp64_single", [d], CH_F64, 2000,
                    note="single 128^2 grid, gamma 0.01, dt 1e-3, noise +-0.1")


def c2() -> Workload:
    d = make_desc((1024, 1024), 0.005, 5e-4, c0=0.0, noise=0.05, seed=2)
    return Workload("ch2d_1024x1024_fp64_single", [d], CH_F64, 20000,
                    note="single 1024^2 grid, gamma 0.005, dt 5e-4, symmetric, noise +-0.05")


def c3(prec: int = CH_F32_BULK, base_seed: int = 1000) -> Workload:
    descs = [make_desc((512, 512), 0.01, 1e-3, c0=(0.0 if m < 32 else 0.3), noise=0.05,
                       seed=base_seed + m) for m in range(64)]
    tag = "fp32" if prec == CH_F32_BULK else "fp64"
    return Workload(f"ch2d_64x512x512_{tag}_ensemble", descs, prec, 10000,
                    note="64 x 512^2, gamma 0.01, dt 1e-3, half C0=0 / half C0=0.3, noise +-0.05")


def c4(meta_seed: int = 4242) -> Workload:
    rng = np.random.default_rng(meta_seed)
    sizes = [256] * 32 + [512] * 16 + [1024] * 4
    descs = []
    for m, n in enumerate(sizes):
        gamma = float(rng.uniform(0.005, 0.02))
        c0 = float(rng.uniform(-0.3, 0.3))
        descs.append(make_desc((n, n), gamma, 5e-4, c0=c0, noise=0.05, seed=4000 + m))
    return Workload("ch2d_mixed_32x256_16x512_4x1024_fp32", descs, CH_F32_BULK, 5000,
                    note="gamma ~ U[0.005,0.02], C0 ~ U[-0.3,0.3] per member, dt 5e-4, noise +-0.05")


def c5() -> Workload:
    descs = [make_desc((256, 256, 256), 0.01, 5e-4, c0=(0.0 if m < 4 else 0.2), noise=0.05,
                       seed=5000 + m) for m in range(8)]
    return Workload("ch3d_8x256cubed_fp32_ensemble", descs, CH_F32_BULK, 5000,
                    note="8 x 256^3, gamma 0.01, dt 5e-4, C0 in {0, 0.2}, noise +-0.05")


def droplet_ic(n: int, eps: float = 1e-6, L: float = TWO_PI) -> np.ndarray:
    """Initial field of the convergence study of Appendix A: a single droplet
    C = eps tanh(r - pi) on the n x n vertex grid x_i = i L / n (numpy order
    (y, x)), with r the distance from the centre of the domain.  (Measured
    from the grid origin, the profile would jump across the periodic
    boundary; centred, it is continuous, and the study then reproduces the
    errors the paper tabulates.)"""
    x = np.arange(n) * (L / n) - L / 2
    X, Y = np.meshgrid(x, x)  # Y varies along axis 0
    return eps * np.tanh(np.sqrt(X * X + Y * Y) - np.pi)


def droplet_steps(n: int, T: float = 10.0, cfl: float = 0.1, L: float = TWO_PI):
    """(nsteps, dt) of the convergence study: dt = cfl * dx rounded so that an
    integer number of steps ends exactly at T."""
    nsteps = int(round(T / (cfl * L / n)))
    return nsteps, T / nsteps


WORKLOADS = {
    "c1": c1,
    "c2": c2,
    "c3": lambda: c3(CH_F32_BULK),
    "c3_fp64": lambda: c3(CH_F64),
    "c4": c4,
    "c5": c5,
}


def get(name: str) -> Workload:
    return WORKLOADS[name]()


def names() -> List[str]:
    return list(WORKLOADS)


# ---- Model 1: droplet populations (Section 3, Table "ensembles") ------------
# M = 100 populations for each N = 128 ... 8192, initial radii i.i.d. U(0, 1)
# (eq. (dRi_init)), statistics over t in [0, 40].
MODEL1_N = (128, 256, 512, 1024, 2048, 4096, 8192)
MODEL1_M = 100
MODEL1_T_END = 40.0


def model1_radii(n: int, seed: int) -> np.ndarray:
    """Initial radii of one population: n draws of U(0, 1), seeded."""
    return np.random.default_rng(seed).uniform(0.0, 1.0, n)


def model1_ensemble(ns=MODEL1_N, M: int = MODEL1_M, base_seed: int = 7000):
    """(sizes, radii) of M populations per size in ns; member m of size index
    k uses seed base_seed + 1000 k + m."""
    sizes, radii = [], []
    for k, n in enumerate(ns):
        for m in range(M):
            sizes.append(int(n))
            radii.append(model1_radii(int(n), base_seed + 1000 * k + m))
    return sizes, radii
