"""Grid-convergence study of the scheme (Appendix A of the paper): the single
droplet C = eps tanh(r - pi) on [0, 2 pi)^2, gamma = 0.01, T = 10,
dt = 0.1 dx, run on successively doubled n x n grids with the library, and

    E_n = (1/|Omega|) integral |C_n - C_{n/2}| dx

between each grid and the one with half the points.  Two ways to match
points are reported:

* "average": the paper's rule, the mean of the 2 x 2 fine points of a coarse
  cell against the coarse point.  On this library's vertex grid
  x_i = i h those fine points are centred h/2 away from the coarse point,
  which alone contributes an O(h) difference;
* "inject": the fine point that coincides with the coarse point.

Runs are FP64 single grids; the comparison is a host-side reduction of the
final fields.
"""
from __future__ import annotations

import math
from typing import Dict, List

import numpy as np

from .ch import CH_F64, Ensemble, make_desc
from .workloads import droplet_ic, droplet_steps


def final_field(n: int, T: float = 10.0, gamma: float = 0.01, eps: float = 1e-6, cfl: float = 0.1,
                prec: int = CH_F64, graph_steps: int = 64) -> np.ndarray:
    """The field at time T on the n x n grid."""
    nsteps, dt = droplet_steps(n, T, cfl)
    ens = Ensemble([make_desc((n, n), gamma, dt)], prec=prec, cadence=nsteps + 1, max_samples=1)
    try:
        ens.set_graph_steps(graph_steps)
        ens.set_field(0, droplet_ic(n, eps))
        ens.step(nsteps)
        return ens.get_field(0)
    finally:
        ens.close()


def difference(fine: np.ndarray, coarse: np.ndarray, match: str) -> float:
    """E_n between a 2n x 2n and an n x n field (mean absolute difference over
    the coarse points, i.e. the integral over |Omega| with the coarse cell
    area as weight)."""
    if match == "average":
        f = 0.25 * (fine[0::2, 0::2] + fine[0::2, 1::2] + fine[1::2, 0::2] + fine[1::2, 1::2])
    elif match == "inject":
        f = fine[0::2, 0::2]
    else:
        raise ValueError(match)
    return float(np.abs(f - coarse).mean())


def study(ns: List[int], **kw) -> List[Dict]:
    """Rows {n, E_average, E_inject, order_average, order_inject} for every n
    of `ns` after the first (E_n compares n with n/2; ns must double)."""
    fields = {n: final_field(n, **kw) for n in ns}
    rows = []
    for a, b in zip(ns, ns[1:]):
        assert b == 2 * a
        rows.append({"n": b, "E_average": difference(fields[b], fields[a], "average"),
                     "E_inject": difference(fields[b], fields[a], "inject")})
    for r, r2 in zip(rows, rows[1:]):
        for m in ("average", "inject"):
            r["order_" + m] = math.log2(r["E_" + m] / r2["E_" + m])
    return rows


if __name__ == "__main__":
    import argparse
    import json

    p = argparse.ArgumentParser()
    p.add_argument("--ns", default="64,128,256,512,1024,2048")
    a = p.parse_args()
    for row in study([int(x) for x in a.ns.split(",")]):
        print(json.dumps(row), flush=True)
