"""The Cahn-Hilliard ensemble statistics of Section 4 (Table "stats_CH",
asymmetric mixtures) at the paper's ensemble size, with the library.

M = 1024 periodic realisations of eq. (ch) with gamma = 0.01 on [0, L)^2,
Delta x = 2 pi / 512 (so n = 512 L / (2 pi)), Delta t = 0.0012, run to
t = 100 from the asymmetric initial condition of Section 4.1,
C = 0.5 + 0.1 (r - 1) with r ~ U(0, 1) i.i.d. per site (mean 0.45, spread
+-0.05).  Reported per L:

* beta0 = (1/80) integral_20^100 mu_1 dt (eq. (beta0_stats), trapezoid rule
  over the recorded samples);
* k, the least-squares slope of mu_2 = k t over the samples in [20, 100]
  (the table's caption);
* bootstrap standard errors of both over the members.

With `symmetric`, the symmetric mixtures of Table "stats_CH_symmetric": the
section's formula C = r has mean 0.5, at odds with a symmetric mixture, and
is read as C = r - 1/2 (c0 = 0, spread +-0.5).  That table's beta0 column is
headed (1/80) int_80^100, so beta0 is reported over both [20, 100] and
[80, 100].

Everything runs on the device (`ch_step`, `ch_ensemble_window`); the host only
resamples member lists for the standard errors.
"""
from __future__ import annotations

import argparse
import math
import os
import time
from typing import Callable, Optional

import numpy as np

from .ch import CH_F32_BULK, CH_F64, Ensemble, make_desc

# Table "stats_CH" of the paper: L / pi -> (beta0, k)
PAPER = {2.0: (0.33, 0.036), 4.0: (0.28, 0.0056), 8.0: (0.28, 0.0013), 16.0: (0.28, 0.00031)}
# Table "stats_CH_symmetric" (L = 2 pi is not reported there)
PAPER_SYMMETRIC = {4.0: (0.356, 0.0011), 8.0: (0.346, 0.00025), 16.0: (0.346, 0.00062)}

_HERE = os.path.dirname(os.path.abspath(__file__))


def run(L_over_pi: float, members: int = 1024, prec: int = CH_F32_BULK, t_end: float = 100.0,
        dt: float = 0.0012, gamma: float = 0.01, cadence: int = 10, seed0: int = 90000, boot: int = 200,
        symmetric: bool = False, tune_cache: Optional[str] = os.path.join(_HERE, "tune_cache.txt"),
        progress: Callable[[str], None] = print) -> dict:
    L = L_over_pi * math.pi
    n = int(round(512 * L / (2 * math.pi)))
    nsteps = int(round(t_end / dt))
    c0, spread = (0.0, 0.5) if symmetric else (0.45, 0.05)
    descs = [make_desc((n, n), gamma, dt, c0=c0, noise=spread, seed=seed0 + m, L=(L, L))
             for m in range(members)]
    ens = Ensemble(descs, prec=prec, cadence=cadence, max_samples=nsteps // cadence + 1)
    try:
        ens.set_graph_steps(64)
        if tune_cache is not None:
            progress(f"L={L_over_pi:g}pi n={n} M={members}: autotuning tiles")
            ens.autotune(tune_cache)
        ens.init_random()
        t0 = time.time()
        chunk = 5000
        done = 0
        while done < nsteps:
            s = min(chunk, nsteps - done)
            ens.step(s)
            done += s
            ens.sync_step()
            progress(f"L={L_over_pi:g}pi n={n} M={members}: step {done}/{nsteps} ({time.time() - t0:.0f} s)")
        wall = time.time() - t0
        beta0, k = ens.ensemble_window(20.0, t_end + 0.5 * dt)
        rng = np.random.default_rng(0)
        bs = np.array([ens.ensemble_window(20.0, t_end + 0.5 * dt, rng.integers(0, members, members))
                       for _ in range(boot)])
        se_b0, se_k = bs.std(axis=0)
        late, se_late = math.nan, math.nan
        if t_end >= 80.0:
            late, _ = ens.ensemble_window(80.0, t_end + 0.5 * dt)
            se_late = float(np.std([ens.ensemble_window(80.0, t_end + 0.5 * dt,
                                                        rng.integers(0, members, members))[0]
                                    for _ in range(boot)]))
        return dict(L_over_pi=L_over_pi, n=n, members=members, steps=nsteps, wall_s=wall,
                    glups=members * n * n * nsteps / wall / 1e9, beta0=beta0, k=k, se_beta0=float(se_b0),
                    se_k=float(se_k), beta0_80_100=late, se_beta0_80_100=se_late,
                    paper=(PAPER_SYMMETRIC if symmetric else PAPER).get(L_over_pi),
                    mixture="symmetric" if symmetric else "asymmetric",
                    prec="f32" if prec == CH_F32_BULK else "f64")
    finally:
        ens.close()


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--L", default="2", help="domain sizes L/pi, comma-separated (paper: 2,4,8,16)")
    ap.add_argument("--members", type=int, default=1024)
    ap.add_argument("--fp64", action="store_true")
    ap.add_argument("--t-end", type=float, default=100.0)
    ap.add_argument("--symmetric", action="store_true", help="symmetric mixtures (c0 = 0, spread +-0.5)")
    args = ap.parse_args()
    for Lp in (float(v) for v in args.L.split(",")):
        r = run(Lp, members=args.members, prec=CH_F64 if args.fp64 else CH_F32_BULK, t_end=args.t_end,
                symmetric=args.symmetric, progress=lambda s: print(s, flush=True))
        print(f"L={Lp:g}pi {r['mixture']}: beta0 [20,100] {r['beta0']:.4f} +- {r['se_beta0']:.4f}, "
              f"[80,100] {r['beta0_80_100']:.4f} +- {r['se_beta0_80_100']:.4f}, "
              f"k {r['k']:.3g} +- {r['se_k']:.2g} (paper {r['paper']}); {r['wall_s']:.1f} s, "
              f"{r['glups']:.1f} GLUPS", flush=True)


if __name__ == "__main__":
    main()
