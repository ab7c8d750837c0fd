"""Pins of the Model 1 oracle (oracle/droplets.py) against facts fixed by the
mathematics rather than by the oracle itself:

* the Dormand-Prince coefficients satisfy the Runge-Kutta order conditions
  (order 5 for the advancing weights, order 4 for the embedded ones), in
  exact rational arithmetic;
* the integrator's global error falls by 2^5 when a fixed step is halved, and
  the embedded estimate's local error by 2^5 (order-4 pair);
* two droplets: the death time and the trajectory of the smaller one, from an
  independent adaptive quadrature of dt/dV (Section 2: with two droplets,
  ubar = 2/(R1+R2) and dV1/dt = 3 (R1-R2)/(R1+R2));
* one droplet, and equal droplets, are stationary (ubar R = 1);
* the total volume sum V_i (dead droplets included) is invariant, since every
  stage's rates sum to zero and Runge-Kutta preserves linear invariants;
* F never increases and beta >= 0 (eq. (dFdt) is a negative sum of squares);
* eq. (dFdt) agrees with a central difference of eq. (Fdef) along the
  trajectory.
"""
from __future__ import annotations

import math
from fractions import Fraction as Fr

import numpy as np
import pytest
from scipy import integrate, optimize

from oracle import droplets as D


def _trees(A, c, b):
    """The Runge-Kutta order conditions up to order 5 as (value, target)."""
    n = len(b)
    Am = [[A[i][j] if j < len(A[i]) else Fr(0) for j in range(n)] for i in range(n)]

    def mv(v):
        return [sum(Am[i][j] * v[j] for j in range(n)) for i in range(n)]

    def dot(w, v):
        return sum(x * y for x, y in zip(w, v))

    one = [Fr(1)] * n
    c2 = [x * x for x in c]
    c3 = [x * x * x for x in c]
    c4 = [x ** 4 for x in c]
    Ac = mv(c)
    Ac2 = mv(c2)
    Ac3 = mv(c3)
    AAc = mv(Ac)
    AAc2 = mv(Ac2)
    AAAc = mv(AAc)
    cAc = [x * y for x, y in zip(c, Ac)]
    conds = [
        (dot(b, one), Fr(1)),
        (dot(b, c), Fr(1, 2)),
        (dot(b, c2), Fr(1, 3)), (dot(b, Ac), Fr(1, 6)),
        (dot(b, c3), Fr(1, 4)), (dot(b, cAc), Fr(1, 8)), (dot(b, Ac2), Fr(1, 12)),
        (dot(b, AAc), Fr(1, 24)),
        (dot(b, c4), Fr(1, 5)), (dot(b, [x * x * y for x, y in zip(c, Ac)]), Fr(1, 10)),
        (dot(b, [x * y for x, y in zip(c, Ac2)]), Fr(1, 15)),
        (dot(b, [x * y for x, y in zip(c, AAc)]), Fr(1, 30)),
        (dot(b, [y * y for y in Ac]), Fr(1, 20)), (dot(b, Ac3), Fr(1, 20)),
        (dot(b, mv(cAc)), Fr(1, 40)), (dot(b, AAc2), Fr(1, 60)), (dot(b, AAAc), Fr(1, 120)),
    ]
    return conds


def test_tableau_order_conditions():
    A, b5, b4, c = D.tableau_exact()
    for i, row in enumerate(A):
        assert sum(row, Fr(0)) == c[i], f"row sum {i}"
    # first same as last: the last stage is evaluated at the order-5 solution
    assert A[6] == b5[:6] and b5[6] == 0
    conds = _trees(A, c, b5)
    assert len(conds) == 17
    for k, (val, want) in enumerate(conds):
        assert val == want, f"order-5 condition {k}"
    for k, (val, want) in enumerate(_trees(A, c, b4)[:8]):
        assert val == want, f"order-4 condition {k}"
    # the embedded weights are not of order 5 (else the estimate would vanish)
    assert any(v != w for v, w in _trees(A, c, b4)[8:])


def _osc(y):
    # y = (u, tau): u' = u cos(tau), tau' = 1; u(t) = exp(sin t)
    return np.array([y[0] * math.cos(y[1]), 1.0])


def test_fixed_step_order_five():
    errs = []
    for h in (0.2, 0.1, 0.05):
        out = {}
        D.dp45(_osc, [1.0, 0.0], 2.0, 2.0, 1e-6, 1e-9, h, on_sample=lambda j, t, y: out.__setitem__(j, y.copy()),
               fixed_h=h)
        errs.append(abs(out[1][0] - math.exp(math.sin(2.0))))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 24 < r1 < 44 and 24 < r2 < 44, (errs, r1, r2)


def test_embedded_estimate_order():
    A, b5, b4, c, e = D.tableau()
    y0 = np.array([1.0, 0.3])

    def one_step(h):
        k = np.zeros((7, 2))
        for s in range(7):
            k[s] = _osc(y0 + h * (A[s, :s] @ k[:s]))
        return h * (e @ k)

    ests = [abs(one_step(h)[0]) for h in (0.1, 0.05, 0.025)]
    assert 24 < ests[0] / ests[1] < 44 and 24 < ests[1] / ests[2] < 44, ests


def test_adaptive_meets_tolerance():
    out = {}
    D.dp45(_osc, [1.0, 0.0], 3.0, 0.5, 1e-9, 1e-12, 1e-3, on_sample=lambda j, t, y: out.__setitem__(j, (t, y.copy())))
    for j, (t, y) in out.items():
        assert t == j * 0.5
        assert abs(y[0] - math.exp(math.sin(t))) < 1e-7


def _two_droplet_time(V, W):
    """t at which the smaller droplet has volume V (starting from V10): the
    integral of dV/(dV1/dt) with dV1/dt = 3 (R1 - R2)/(R1 + R2)."""
    def g(v):
        r1, r2 = np.cbrt(v), np.cbrt(W - v)
        return (r1 + r2) / (3.0 * (r2 - r1))
    return g


def test_two_droplets_against_quadrature():
    R0 = np.array([0.6, 0.9])
    V0 = D.volumes_from_radii(R0)
    W = float(V0.sum())
    g = _two_droplet_time(None, W)
    tstar = integrate.quad(g, 0.0, V0[0], epsabs=1e-13, epsrel=1e-13, limit=200)[0]
    dts = 0.01
    t_end = round((tstar + 0.3) / dts) * dts
    got = {}
    D.dp45(D.rate, V0, t_end, dts, 1e-10, 1e-13, 1e-4,
           on_sample=lambda j, t, y: got.__setitem__(j, y.copy()))
    checked = 0
    for j, y in sorted(got.items()):
        t = j * dts
        if t < tstar - 0.02:
            # V1(t): invert t(V) = int_V^V10 g
            v = optimize.brentq(lambda v: integrate.quad(g, v, V0[0], epsabs=1e-14, epsrel=1e-13)[0] - t,
                                0.0, V0[0], xtol=1e-15)
            assert abs(y[0] - v) < 1e-8, (t, y[0], v)
            assert y[0] > 0
            checked += 1
        elif t > tstar + 0.02:
            assert y[0] <= 0.0  # dead
            assert abs(y[1] - W) < 1e-9  # the survivor holds the whole volume
    assert checked > 20
    # |dV1/dt| grows from 3 (R2-R1)/(R1+R2) at t = 0 to 3 at death
    assert V0[0] / 3.0 < tstar < V0[0] / (3.0 * (0.9 - 0.6) / 1.5)


def test_stationary_states():
    for R0 in ([0.7], [0.7] * 5):
        s, V, acc, rej = D.run_member(R0, 1.0, dts=0.25)
        assert np.max(np.abs(V - D.volumes_from_radii(R0))) < 1e-14
        assert np.all(np.abs(s[:, 2]) < 1e-13)  # dF/dt
        assert np.all(s[:, 5] == len(R0))


def _radii(n, seed, lo=0.0, hi=1.0):
    return np.random.default_rng(seed).uniform(lo, hi, n)


def test_volume_invariant_energy_decay_and_beta_sign():
    R0 = _radii(300, 11)
    got = []
    s = np.full((21, 6), np.nan)

    def rec(j, t, y):
        got.append(float(np.sum(y)))
        s[j] = D.diagnostics(t, y)

    D.dp45(D.rate, D.volumes_from_radii(R0), 2.0, 0.1, 1e-6, 1e-9, 1e-4, on_sample=rec)
    tot = np.array(got)
    assert np.max(np.abs(tot - tot[0])) < 1e-12 * tot[0]
    assert np.all(np.diff(s[:, 1]) <= 0.0)  # F non-increasing
    assert s[0, 3] == 0.0 and np.all(s[1:, 3] > 0.0)  # beta
    assert np.all(np.diff(s[:, 5]) <= 0.0) and s[-1, 5] < 300  # droplets die, none revive


def test_dFdt_matches_difference_of_F():
    R0 = _radii(40, 5, 0.8, 1.2)
    s, _, _, _ = D.run_member(R0, 0.05, dts=1e-3, rtol=1e-12, atol=1e-14)
    assert np.all(s[:, 5] == 40)  # nobody dies in this window
    fd = (s[2:, 1] - s[:-2, 1]) / (2e-3)
    rel = np.abs(fd - s[1:-1, 2]) / np.abs(s[1:-1, 2])
    assert np.max(rel) < 1e-5, np.max(rel)


# --------------------------------------------------------------------------
# The radius form of Section 3.1 against the volume form
# --------------------------------------------------------------------------
def test_radius_form_matches_volume_form_before_first_death():
    """Where both are defined (before any droplet reaches R = 0) the radius
    form dR/dt = -1/R^2 + ubar/R and the volume form dV/dt = 3 (ubar R - 1)
    are the same law: at tight tolerances their series and states agree to
    the integrators' error."""
    rng = np.random.default_rng(11)
    R0 = rng.uniform(0.45, 1.0, 32)
    s, _, _, _ = D.run_member(R0, 1.0, dts=0.01, rtol=1e-11, atol=1e-14)
    t_death = s[np.argmax(s[:, 5] < 32), 0]
    assert 0.05 < t_death < 1.0
    T = 0.8 * t_death
    sv, V, _, _ = D.run_member(R0, T, dts=T / 20, rtol=1e-11, atol=1e-14)
    sr, R, _, _ = D.run_member_radius(R0, T, dts=T / 20, rtol=1e-11, atol=1e-14, norm="max")
    assert np.all(sr[:, 5] == 32) and np.all(sv[:, 5] == 32)
    for col in (1, 2, 4):
        assert np.abs(sr[:, col] - sv[:, col]).max() <= 1e-9 * np.abs(sv[:, col]).max(), col
    assert np.abs(sr[1:, 3] - sv[1:, 3]).max() <= 1e-8
    assert np.abs(R - np.cbrt(V)).max() <= 1e-9


def test_radius_form_death_and_regularisation():
    """A droplet that reaches R = 0 leaves the mean field and the energy at
    the same sample as in the volume form, then runs on to R <= -eps and
    stops; F of the two forms agrees to the loose tolerance's error."""
    R0 = np.array([0.5, 0.9, 1.0])
    sv, V, _, _ = D.run_member(R0, 1.0, dts=0.01, rtol=1e-11, atol=1e-14)
    sr, R, _, _ = D.run_member_radius(R0, 1.0, dts=0.01, rtol=1e-3, atol=1e-6, norm="rms")
    np.testing.assert_array_equal(sr[:, 5], sv[:, 5])
    assert sv[-1, 5] == 2.0 and V[0] <= 0.0
    assert R[0] <= -D.EPS_RADIUS and R[1] > 0 and R[2] > 0
    assert np.abs(sr[:, 1] - sv[:, 1]).max() <= 1e-5 * sv[0, 1]
    # after the death the diagnostics see the two live droplets only
    assert sr[-1, 1] == pytest.approx(0.5 * (R[1] ** 2 + R[2] ** 2), rel=1e-15)


def test_radius_form_needs_the_rms_norm():
    """With ode45's max norm the singular rate at R = 0 stops the integration
    at the first death of a U(0, 1) population (the step size underflows);
    the root-mean-square norm passes it at rtol 1e-3 but not at 1e-5."""
    R0 = np.random.default_rng(123).uniform(0.0, 1.0, 64)
    with pytest.raises(FloatingPointError):
        D.run_member_radius(R0, 40.0, rtol=1e-3, atol=1e-6, norm="max")
    s, _, _, _ = D.run_member_radius(R0, 40.0, rtol=1e-3, atol=1e-6, norm="rms")
    assert np.all(np.isfinite(s[:, 1])) and s[-1, 5] >= 1
    with pytest.raises(FloatingPointError):
        D.run_member_radius(R0, 40.0, rtol=1e-5, atol=1e-8, norm="rms")


def test_beta_from_F_differences_definition():
    t = np.linspace(0.0, 1.0, 11)
    F = 2.0 * (1.0 + t) ** -0.5  # beta = t / (2 (1 + t)) exactly for this F
    s = np.zeros((11, 6))
    s[:, 0], s[:, 1] = t, F
    b = D.beta_from_F_differences(s)
    exact = t / (2.0 * (1.0 + t))
    assert b[0] == 0.0 and np.abs(b[1:-1] - exact[1:-1]).max() < 2e-3
