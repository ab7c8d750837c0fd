"""Convergence study of Appendix A on the GPU: the final fields against the
oracle at small n, E_n against the oracle's, the paper's table, and first
order at larger n.

The droplet starts at amplitude 1e-6 and grows by spinodal instability, so
rounding differences are amplified along the run.  The parity bar is set by
that amplification, measured on the oracle itself: the droplet field is
symmetric under x <-> y and the x and y factors of the scheme commute, so the
oracle run on the transposed field differs from the direct run only by
rounding order.  The GPU must agree with the oracle within 10x that spread
(plus 1e-12).  Parity is checked at n = 128 and 256, where the interface is
resolved: at n = 64 (grid spacing 0.7 interface widths) the run passes an
unstable event near t = 5 that amplifies differences of 1e-14 a thousand
billion times, and the GPU and oracle fields part there (measured once:
6e-14 at step 400, 0.48 at step 1019)."""
import os

import numpy as np
import pytest

import oracle
from oracle import convergence as oconv
from paper_1911_03386_amd import convergence as conv
from paper_1911_03386_amd import workloads

pytestmark = pytest.mark.gpu


def test_final_fields_and_errors_vs_oracle():
    F, R = {}, {}
    for n in (128, 256):
        nsteps, dt = workloads.droplet_steps(n)
        C0 = workloads.droplet_ic(n)
        F[n] = conv.final_field(n)
        R[n] = oracle.step(C0, 0.01, dt, nsteps)
        spread = float(np.abs(oracle.step(C0.T.copy(), 0.01, dt, nsteps).T - R[n]).max())
        err = float(np.abs(F[n] - R[n]).max())
        print(f"droplet n={n}: {nsteps} steps, max |C - oracle| = {err:.3e}, "
              f"oracle rounding-order spread {spread:.3e}")
        assert err <= 10 * spread + 1e-12
    for m in ("average", "inject"):
        e, r = conv.difference(F[256], F[128], m), oconv.difference(R[256], R[128], m)
        print(f"E_256 ({m}): GPU {e:.6e}, oracle {r:.6e}")
        assert abs(e - r) <= 1e-6 * r, (m, e, r)


def _paper_table():
    rows = {}
    path = os.path.join(os.path.dirname(__file__), "golden", "convergence_table_appendixA.txt")
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            n, e = line.split()
            rows[int(n)] = float(e)
    return rows


def test_convergence_table_and_first_order():
    """Appendix A, Table tab:cvg, at n = 512 .. 2048 (2 x 2 averaging) to
    15 %, as the oracle matches it at n = 128, 256; the averaged error falls
    at first order, as the paper reports."""
    table = _paper_table()
    rows = conv.study([256, 512, 1024, 2048])
    for r in rows:
        print({k: round(v, 6) if isinstance(v, float) else v for k, v in r.items()},
              "paper", table.get(r["n"]))
        assert abs(r["E_average"] / table[r["n"]] - 1) <= 0.15, r
    assert 0.8 <= rows[-2]["order_average"] <= 1.3


def test_convergence_e4096_against_the_table():
    """Appendix A, Table tab:cvg: E_4096, the 4096^2 grid (65190 steps of
    16.7 M sites) against the 2048^2 one, to 15 % with 2 x 2 averaging."""
    table = _paper_table()
    (r,) = conv.study([2048, 4096])
    print({k: round(v, 7) if isinstance(v, float) else v for k, v in r.items()}, "paper", table[4096])
    assert abs(r["E_average"] / table[4096] - 1) <= 0.15, r
