"""The stored Model 1 study (tests/golden/model1_radius_form_study.txt,
written by tests/golden/model1_radius_form_study.py from the oracle alone):
its rows are reproducible (population 0 of each cheap row recomputed), and
the facts the study establishes are asserted here:

* the paper's regularised radius form, integrated with the Dormand-Prince
  pair under root-mean-square error control at rtol 1e-3 (the loosest
  setting, where it passes every death), gives the same beta0 as the volume
  form the library integrates (N = 512: within a quarter of a standard
  error): the regularisation is result-neutral, as Section 3.1 says of eps;
* it stops at the first death under ode45's max norm, and under the RMS norm
  once rtol is tight enough (the step size underflows at R = 0).
"""
import os

import numpy as np
import pytest

from oracle import droplets as D
from paper_1911_03386_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "model1_radius_form_study.txt")
TABLE_NS = (512, 1024, 2048, 4096, 8192)


def study_rows():
    rows = []
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        f = line.split()
        rows.append(dict(N=int(f[0]), form=f[1], norm=f[2], rtol=float(f[3]), atol=float(f[4]), beta=f[5],
                         completed=int(f[6]), b0=float(f[7]), se_b0=float(f[8]), k=float(f[9]),
                         se_k=float(f[10]), F40=float(f[11]), beta40=float(f[12])))
    return rows


def row(N, form, norm, rtol, beta):
    for r in study_rows():
        if (r["N"], r["form"], r["norm"], r["beta"]) == (N, form, norm, beta) and np.isclose(r["rtol"], rtol):
            return r
    raise KeyError((N, form, norm, rtol, beta))


def population0(N):
    sizes, radii = W.model1_ensemble(ns=TABLE_NS)
    return radii[sizes.index(N)]


@pytest.mark.parametrize("form,rtol,atol,beta", [("volume", 1e-6, 1e-9, "identity"),
                                                 ("radius", 1e-3, 1e-6, "Fdiff")])
def test_study_rows_reproduce(form, rtol, atol, beta):
    r = row(512, form, "max" if form == "volume" else "rms", rtol, beta)
    R0 = population0(512)
    if form == "volume":
        ser, _, _, _ = D.run_member(R0, 40.0, 0.1, rtol, atol)
        b = ser[:, 3]
    else:
        ser, _, _, _ = D.run_member_radius(R0, 40.0, 0.1, rtol, atol, norm="rms")
        b = D.beta_from_F_differences(ser)
    assert ser[-1, 1] == pytest.approx(r["F40"], rel=1e-9)
    assert b[-1] == pytest.approx(r["beta40"], rel=1e-6, abs=1e-12)


def test_radius_form_is_result_neutral_at_n512():
    v = row(512, "volume", "max", 1e-6, "identity")
    rf = row(512, "radius", "rms", 1e-3, "Fdiff")
    ri = row(512, "radius", "rms", 1e-3, "identity")
    assert v["completed"] == rf["completed"] == 100
    assert abs(rf["b0"] - v["b0"]) <= 0.25 * v["se_b0"], (rf, v)
    assert abs(ri["b0"] - v["b0"]) <= 0.5 * v["se_b0"], (ri, v)


def test_radius_form_stops_where_the_study_says():
    assert row(512, "radius", "max", 1e-3, "Fdiff")["completed"] == 0
    assert row(512, "radius", "rms", 1e-5, "Fdiff")["completed"] < 100
