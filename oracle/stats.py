"""Ensemble statistics of the coarsening rate: plain definitions in FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring): the parity reference for
the library's device-side ensemble statistics.  Inputs are the oracle's own
beta series (``oracle.run_series``), never values from the HIP path.

Definitions (Sections 3.3 and 4 of the paper):

* eq. (mup): over M members at each sample time,
  mu_1 = (1/M) sum_j beta_j,   mu_p = (1/M) sum_j (beta_j - mu_1)^p, p >= 2;
* eq. (beta0_stats): beta0 = (1/(t2 - t1)) integral_{t1}^{t2} mu_1 dt, read here
  as the trapezoid rule over the recorded samples with t1 <= t <= t2, divided by
  the time those samples span;
* the variance trend E(dbeta^2) = k t: k is the least-squares slope of mu_2
  against t through the origin over the same samples,
  k = sum t mu_2 / sum t^2;
* time-resolved histograms of beta: counts of beta_j(t) over the members and
  the window's samples in nbins equal bins of [lo, hi), plus the counts below
  lo and at or above hi.  A value's bin is floor((beta - lo) * (nbins / (hi -
  lo))) in FP64, capped at nbins - 1.
"""
from __future__ import annotations

import math

import numpy as np


def ensemble_moments(beta: np.ndarray, pmax: int) -> np.ndarray:
    """beta: (M, J) per member and sample.  Returns (J, pmax): column 0 is
    mu_1, column p-1 is mu_p (eq. (mup)); sums are exactly rounded."""
    beta = np.asarray(beta, dtype=np.float64)
    M, J = beta.shape
    out = np.empty((J, pmax))
    for j in range(J):
        col = [float(b) for b in beta[:, j]]
        mu1 = math.fsum(col) / M
        out[j, 0] = mu1
        for p in range(2, pmax + 1):
            out[j, p - 1] = math.fsum((b - mu1) ** p for b in col) / M
    return out


def window_samples(t: np.ndarray, t1: float, t2: float):
    """Indices of the recorded samples with t1 <= t <= t2."""
    return [j for j, tj in enumerate(t) if t1 <= tj <= t2]


def ensemble_window(t: np.ndarray, mu1: np.ndarray, mu2: np.ndarray, t1: float, t2: float):
    """(beta0, k) over the samples in [t1, t2]: the trapezoid time average of
    mu_1 (eq. (beta0_stats)) and the slope of mu_2 = k t through the origin."""
    idx = window_samples(t, t1, t2)
    if not idx:
        return math.nan, math.nan
    area = math.fsum(0.5 * (t[j + 1] - t[j]) * (mu1[j] + mu1[j + 1]) for j in idx[:-1])
    span = t[idx[-1]] - t[idx[0]]
    beta0 = area / span if len(idx) > 1 else math.nan
    num = math.fsum(t[j] * mu2[j] for j in idx)
    den = math.fsum(t[j] * t[j] for j in idx)
    k = num / den if den > 0 else math.nan
    return beta0, k


def beta_histogram(beta: np.ndarray, t: np.ndarray, t1: float, t2: float, lo: float, hi: float,
                   nbins: int) -> np.ndarray:
    """Counts [below lo, bins 1..nbins over [lo, hi), at or above hi] of beta
    over all members and the samples in [t1, t2]; NaN is not counted."""
    counts = np.zeros(nbins + 2, dtype=np.int64)
    scale = nbins / (hi - lo)
    for j in window_samples(t, t1, t2):
        for b in np.asarray(beta)[:, j]:
            b = float(b)
            if math.isnan(b):
                continue
            if b < lo:
                counts[0] += 1
            elif b >= hi:
                counts[nbins + 1] += 1
            else:
                counts[1 + min(nbins - 1, int((b - lo) * scale))] += 1
    return counts
