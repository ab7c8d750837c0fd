"""Grid-convergence error of Appendix A, written out with loops.

TEST INFRASTRUCTURE ONLY (see the package docstring).  E_n between a 2n x 2n
and an n x n field: (1/|Omega|) sum over the coarse points of |fine value -
coarse value| times the coarse cell area, with the fine value either the mean
of the 2 x 2 fine points of the coarse cell (the paper's rule) or the fine
point at the coarse point ("inject")."""
from __future__ import annotations

import math

import numpy as np


def difference(fine: np.ndarray, coarse: np.ndarray, match: str) -> float:
    n = coarse.shape[0]
    assert coarse.shape == (n, n) and fine.shape == (2 * n, 2 * n)
    terms = []
    for j in range(n):
        for i in range(n):
            if match == "average":
                f = 0.25 * (fine[2 * j, 2 * i] + fine[2 * j, 2 * i + 1] + fine[2 * j + 1, 2 * i]
                            + fine[2 * j + 1, 2 * i + 1])
            else:
                f = fine[2 * j, 2 * i]
            terms.append(abs(float(f) - float(coarse[j, i])))
    # cell area (2 pi / n)^2 over |Omega| = (2 pi)^2: the mean
    return math.fsum(terms) / (n * n)
