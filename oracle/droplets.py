"""Model 1 (mean-field droplet population) in plain FP64: the reference.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline of the benchmark use this module; the library never imports it and
shares no code with it.

What it computes (paper, Section 2, eq. (dRi) with eq. (uval); Section 3.1,
the regularised form of eq. (dRi); Section 2.3, eq. (Fdef), eq. (dFdt) and
eq. (betaN)):

* N droplets with radii R_i.  A droplet is alive while R_i > 0 (the Heaviside
  factor H(R_i)) and obeys  dR_i/dt = -1/R_i^2 + ubar/R_i,  with the mean
  field  ubar = sum_i H(R_i) / sum_i H(R_i) R_i.  The initial radii are drawn
  from U(0, 1) (eq. (dRi_init)); here they are an input.
* The state integrated is the volume V_i = R_i^3 (up to 4 pi / 3), for which
  the same law reads  dV_i/dt = 3 (ubar R_i - 1),  R_i = V_i^(1/3).  It is
  bounded where dR/dt is singular: a droplet reaches V = 0 at a finite speed
  and is dead from then on (its rate is 0 while V <= 0).  This is the paper's
  regularisation H(R + eps) in the limit eps -> 0, which the paper reports
  does not change its results.  V_i = (R_i R_i) R_i at t = 0.
* Time stepping: the explicit Runge-Kutta pair of Dormand and Prince (1980),
  order 5 with an embedded order-4 estimate, advancing with the order-5
  solution (the pair inside MATLAB's ode45, which the paper used), with
  error control
      err = max_i |h sum_s e_s k_{s,i}| / (atol + rtol max(|V_i|, |V_i^new|)),
      e = b(5) - b(4);
  accepted iff err <= 1.  Step-size update: factor = 0.9 err^(-1/5) clamped
  to [0.2, 5] (5 when err = 0), after a rejection no growth on the next
  accepted step.  A step that would pass the next sample time t_j = j dts is
  shortened to end exactly on it.
* Samples (t_j = j dts, j = 0..J-1) of the state: F = (1/2) sum H R^2
  (eq. (Fdef) once the volume constraint holds), dF/dt = -sum H (1/R)
  (1 - ubar R)^2 (eq. (dFdt)), beta = -t (dF/dt) / F (eq. (betaN)), ubar and
  the number of live droplets.

Sums over droplets inside a step use numpy's pairwise sum; the sample
diagnostics use exactly rounded sums (math.fsum).

The radius form (Section 3.1 as printed) is here too, for the comparison with
the paper's own runs: the state is R itself and

    dR_i/dt = H(R_i + eps) (-1/R_i^2 + ubar/R_i),  ubar over the R_i > 0,

eps = 1e-3: a droplet that crosses R = 0 leaves the mean field and the
energy at once and keeps moving (ever faster) until R <= -eps, where it
stops.  The rate is singular at R = 0, so an integrator has to shrink its
step there; with the max norm above it cannot pass the first death (the step
underflows), while the root-mean-square norm
    err = sqrt(mean_i (|h sum_s e_s k_{s,i}| / (atol + rtol max(|R_i|, |R_i^new|)))^2)
(Hairer, Norsett and Wanner's choice) dilutes one droplet's error over the
population and lets loose tolerances through.  The same integrator serves
both forms (`norm` selects the error norm).
"""
from __future__ import annotations

import math
from fractions import Fraction as Fr

import numpy as np

SLOTS = ("t", "F", "dFdt", "beta", "ubar", "alive")

# Dormand & Prince (1980), the 7-stage FSAL pair; exact rationals.
_A = [
    [],
    [Fr(1, 5)],
    [Fr(3, 40), Fr(9, 40)],
    [Fr(44, 45), Fr(-56, 15), Fr(32, 9)],
    [Fr(19372, 6561), Fr(-25360, 2187), Fr(64448, 6561), Fr(-212, 729)],
    [Fr(9017, 3168), Fr(-355, 33), Fr(46732, 5247), Fr(49, 176), Fr(-5103, 18656)],
    [Fr(35, 384), Fr(0), Fr(500, 1113), Fr(125, 192), Fr(-2187, 6784), Fr(11, 84)],
]
_B5 = [Fr(35, 384), Fr(0), Fr(500, 1113), Fr(125, 192), Fr(-2187, 6784), Fr(11, 84), Fr(0)]
_B4 = [Fr(5179, 57600), Fr(0), Fr(7571, 16695), Fr(393, 640), Fr(-92097, 339200), Fr(187, 2100),
       Fr(1, 40)]
_C = [Fr(0), Fr(1, 5), Fr(3, 10), Fr(4, 5), Fr(8, 9), Fr(1), Fr(1)]


def tableau_exact():
    """(A, b5, b4, c) of the Dormand-Prince pair as Fractions; A is lower
    triangular, row s holding a_{s,0..s-1}."""
    return [list(r) for r in _A], list(_B5), list(_B4), list(_C)


def tableau():
    """The same pair in FP64: A (7x7), b5, b4, c, e = b5 - b4."""
    A = np.zeros((7, 7))
    for s, row in enumerate(_A):
        for j, v in enumerate(row):
            A[s, j] = float(v)
    b5 = np.array([float(v) for v in _B5])
    b4 = np.array([float(v) for v in _B4])
    c = np.array([float(v) for v in _C])
    e = np.array([float(x - y) for x, y in zip(_B5, _B4)])
    return A, b5, b4, c, e


def _step_factor(err: float) -> float:
    if err == 0.0:
        return 5.0
    return min(5.0, max(0.2, 0.9 * err ** -0.2))


def dp45(f, y0, t_end: float, dts: float, rtol: float, atol: float, h0: float,
         max_attempts: int = 10**7, on_sample=None, fixed_h: float | None = None, norm: str = "max"):
    """Integrate y' = f(y) (autonomous, vector y) from t = 0 with the
    Dormand-Prince pair and the error control above.  Samples at t_j = j dts,
    j = 0..J-1 with J = round(t_end/dts) + 1: on_sample(j, t_j, y) is called
    on each (also j = 0).  With fixed_h, every step is accepted with that
    size (sample clipping still applies).  norm: "max" (the default, as
    ode45) or "rms" over the components.  Returns (y, accepted, rejected)."""
    if norm not in ("max", "rms"):
        raise ValueError(norm)
    A, b5, _, _, e = tableau()
    J = int(round(t_end / dts)) + 1
    y = np.array(y0, dtype=np.float64)
    t, h, jn = 0.0, float(fixed_h if fixed_h is not None else h0), 1
    rejected_last = False
    acc = rej = 0
    if on_sample is not None:
        on_sample(0, 0.0, y)
    k = np.zeros((7,) + y.shape)
    while jn < J:
        if acc + rej >= max_attempts:
            raise RuntimeError("step limit reached")
        t_next = jn * dts
        land = h >= t_next - t
        if land:
            h = t_next - t
        for s in range(7):
            incr = np.zeros_like(y)
            for j in range(s):
                incr = incr + A[s, j] * k[j]
            k[s] = f(y + h * incr)
        incr = np.zeros_like(y)
        for j in range(6):
            incr = incr + b5[j] * k[j]
        y5 = y + h * incr
        est = np.zeros_like(y)
        for j in range(7):
            est = est + e[j] * k[j]
        sc = atol + rtol * np.maximum(np.abs(y), np.abs(y5))
        q = np.abs(h * est) / sc
        if not y.size:
            err = 0.0
        elif norm == "max":
            err = float(np.max(q))
        else:
            err = math.sqrt(float(np.mean(q * q)))
        if not math.isfinite(err):
            raise FloatingPointError("non-finite error estimate")
        if fixed_h is not None:
            err = 0.0
        if err <= 1.0:
            y = y5
            t = t_next if land else t + h
            fac = _step_factor(err)
            if rejected_last:
                fac = min(fac, 1.0)
            rejected_last = False
            acc += 1
            if fixed_h is not None:
                h = float(fixed_h)
            else:
                h = h * fac
            if land:
                if on_sample is not None:
                    on_sample(jn, t, y)
                jn += 1
        else:
            h = h * max(0.2, 0.9 * err ** -0.2)
            rejected_last = True
            rej += 1
        if jn < J and t + h == t:
            raise FloatingPointError("step size underflow")
    return y, acc, rej


def volumes_from_radii(R0) -> np.ndarray:
    """V = (R R) R, the integrated state at t = 0."""
    R0 = np.asarray(R0, dtype=np.float64)
    return (R0 * R0) * R0


def mean_field(V: np.ndarray) -> float:
    """ubar = sum H / sum H R over the live droplets (eq. (uval)); 0 when none
    is alive (then every rate is 0 anyway)."""
    alive = V > 0.0
    cnt = int(np.count_nonzero(alive))
    if cnt == 0:
        return 0.0
    return cnt / float(np.sum(np.cbrt(V[alive])))


def rate(V: np.ndarray) -> np.ndarray:
    """dV/dt = 3 (ubar R - 1) for live droplets, 0 for dead ones, with ubar of
    eq. (uval) (the same sum as mean_field)."""
    alive = V > 0.0
    R = np.where(alive, np.cbrt(np.where(alive, V, 1.0)), 0.0)
    cnt = int(np.count_nonzero(alive))
    ubar = cnt / float(np.sum(R[alive])) if cnt else 0.0
    return np.where(alive, 3.0 * (ubar * R - 1.0), 0.0)


def _diagnostics_of_radii(t: float, R):
    n = len(R)
    if n == 0:
        return (t, 0.0, 0.0, math.nan, 0.0, 0.0)
    ubar = n / math.fsum(R)
    F = 0.5 * math.fsum(r * r for r in R)
    dF = -math.fsum((1.0 - ubar * r) ** 2 / r for r in R)
    beta = 0.0 if t == 0.0 else -t * dF / F
    return (t, F, dF, beta, ubar, float(n))


def diagnostics(t: float, V: np.ndarray):
    """(t, F, dF/dt, beta, ubar, alive) of a state, exactly rounded sums."""
    alive = V > 0.0
    return _diagnostics_of_radii(t, [float(r) for r in np.cbrt(V[alive])])


def run_member(R0, t_end: float, dts: float = 0.1, rtol: float = 1e-6, atol: float = 1e-9,
               h0: float = 1e-4, max_attempts: int = 10**7):
    """One member from radii R0: returns (series (J, 6) in SLOTS order, final
    V, accepted steps, rejected steps)."""
    J = int(round(t_end / dts)) + 1
    series = np.full((J, len(SLOTS)), np.nan)

    def rec(j, t, y):
        series[j] = diagnostics(t, y)

    V, acc, rej = dp45(rate, volumes_from_radii(R0), t_end, dts, rtol, atol, h0, max_attempts, rec)
    return series, V, acc, rej


# --------------------------------------------------------------------------
# The radius form of Section 3.1 (the paper's own numerics)
# --------------------------------------------------------------------------
EPS_RADIUS = 1e-3  # the paper's eps


def rate_radius(R: np.ndarray, eps: float = EPS_RADIUS) -> np.ndarray:
    """dR/dt = H(R + eps) (-1/R^2 + ubar/R) with ubar = sum H(R) / sum H(R) R
    (eq. (uval)); 0 where R <= -eps."""
    alive = R > 0.0
    cnt = int(np.count_nonzero(alive))
    ubar = cnt / float(np.sum(R[alive])) if cnt else 0.0
    moving = R > -eps
    Rs = np.where(moving & (R != 0.0), R, 1.0)
    return np.where(moving & (R != 0.0), -1.0 / (Rs * Rs) + ubar / Rs, np.where(moving, -np.inf, 0.0))


def diagnostics_radius(t: float, R: np.ndarray):
    """(t, F, dF/dt, beta, ubar, alive) of a radius state: the droplets with
    R > 0 (H(R)), eq. (Fdef), eq. (dFdt), eq. (betaN); exactly rounded sums."""
    return _diagnostics_of_radii(t, [float(r) for r in R[R > 0.0]])


def run_member_radius(R0, t_end: float, dts: float = 0.1, rtol: float = 1e-3, atol: float = 1e-6,
                      h0: float = 1e-4, eps: float = EPS_RADIUS, norm: str = "rms",
                      max_attempts: int = 10**7):
    """One member in the radius form: returns (series (J, 6) in SLOTS order,
    final R, accepted, rejected).  Raises FloatingPointError when the step
    size underflows (at a death, for tight tolerances or the max norm)."""
    J = int(round(t_end / dts)) + 1
    series = np.full((J, len(SLOTS)), np.nan)

    def rec(j, t, y):
        series[j] = diagnostics_radius(t, y)

    R, acc, rej = dp45(lambda y: rate_radius(y, eps), np.array(R0, dtype=np.float64), t_end, dts, rtol, atol,
                       h0, max_attempts, rec, norm=norm)
    return series, R, acc, rej


def beta_from_F_differences(series: np.ndarray) -> np.ndarray:
    """beta_j = -t_j (F_{j+1} - F_{j-1}) / ((t_{j+1} - t_{j-1}) F_j) from the
    sampled F (one-sided at the ends; 0 at t = 0): the coarsening rate of
    eq. (betaN) with dF/dt taken from the output grid."""
    t, F = series[:, 0], series[:, 1]
    dF = np.empty_like(F)
    dF[1:-1] = (F[2:] - F[:-2]) / (t[2:] - t[:-2])
    dF[0] = (F[1] - F[0]) / (t[1] - t[0])
    dF[-1] = (F[-1] - F[-2]) / (t[-1] - t[-2])
    beta = -t * dF / F
    beta[0] = 0.0
    return beta
