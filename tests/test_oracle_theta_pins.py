"""Pins of the oracle's Crank-Nicolson ADI variant (theta = 1/2):

    prod_d (I + gamma dt D_d^2 / 2) C^{n+1}
        = prod_d (I - gamma dt D_d^2 / 2) C^n + dt lap_h(C^3 - C) - 2 gamma dt sum_{d<e} D_d D_e C^n

checked against what the mathematics fixes: the closed-form growth factor of
single Fourier modes, second order in dt where only the pure fourth
derivatives act (Appendix A: the scheme for hyper-diffusion alone is second
order) against the spatially discrete flow integrated to high accuracy, first
order once the explicit mixed term enters, conservation of <C> and the odd
symmetry."""
import numpy as np
import pytest

from tests import refs

TWO_PI = 2 * np.pi
C_FLAT = 1.0 / np.sqrt(3.0)  # 3 C0^2 - 1 = 0: the linearised flow is pure hyper-diffusion


@pytest.mark.parametrize("k,c0,tol", [((5, 0), 0.0, 1e-12), ((5, 5), 0.0, 1e-12),
                                     ((20, 20), 0.0, 1e-12), ((40, 7), 0.0, 1e-12),
                                     ((64, 0), 0.0, 1e-12), ((5, 5), 0.3, 1e-8), ((11, 3), 0.3, 1e-8)])
def test_theta_half_single_mode_amplification(orc, k, c0, tol):
    n, gamma, dt, eps = 128, 0.01, 1e-3, 1e-7
    x = np.arange(n) * TWO_PI / n
    X, Y = np.meshgrid(x, x, indexing="xy")
    mode = np.cos(k[0] * X + k[1] * Y)
    C1 = orc.step(c0 + eps * mode, gamma, dt, 1, theta=0.5)
    G = np.sum((C1 - c0) * mode) / np.sum(mode * mode) / eps
    Gh = refs.amplification(k, (n, n), TWO_PI, gamma, dt, c0, theta=0.5)
    assert abs(G - Gh) <= tol * max(1.0, abs(Gh)), (G, Gh)


def test_theta_half_3d_single_mode(orc):
    n, gamma, dt, eps, k = 16, 0.01, 5e-4, 1e-7, (2, 3, 1)
    x = np.arange(n) * TWO_PI / n
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    mode = np.cos(k[0] * X + k[1] * Y + k[2] * Z)
    C1 = orc.step(eps * mode, gamma, dt, 1, theta=0.5)
    G = np.sum(C1 * mode) / np.sum(mode * mode) / eps
    assert abs(G - refs.amplification(k, (n, n, n), TWO_PI, gamma, dt, 0.0, theta=0.5)) < 1e-12


def test_theta_half_grid_scale_mode_not_damped(orc):
    """The stiff axis modes of Crank-Nicolson have growth factors near -1: at
    rho = gamma dt / h^4 = 441 (512^2, dt = 1e-3) the grid-scale x mode keeps
    99 % of its amplitude per step and flips sign (theta = 1 leaves 0.4 %)."""
    n, gamma, dt = 512, 0.01, 1e-3
    Gh = refs.amplification((n // 2, 0), (n, n), TWO_PI, gamma, dt, 0.0, theta=0.5)
    G1 = refs.amplification((n // 2, 0), (n, n), TWO_PI, gamma, dt, 0.0)
    assert -1.0 < Gh < -0.99 and 0 < G1 < 5e-3
    x = np.zeros((8, n))
    x[:, ::2], x[:, 1::2] = 1e-7, -1e-7  # the mode itself (y-invariant)
    C1 = orc.step(x, gamma, dt, 1, theta=0.5)
    assert abs(C1[0, 0] / 1e-7 - Gh) < 1e-9


def _order_study(orc, C0, gamma, T, dts, theta):
    ref = refs.semi_discrete_flow(C0, gamma, T, 1e-3)
    errs = []
    for dt in dts:
        C = orc.step(C0, gamma, dt, int(round(T / dt)), theta=theta)
        errs.append(float(np.abs(C - ref).max()))
    return errs


def _modes_x(n, ny, ks, amp, seed=3):
    rng = np.random.default_rng(seed)
    x = np.arange(n) * TWO_PI / n
    row = sum(np.cos(k * x + rng.uniform(0, TWO_PI)) for k in ks)
    return C_FLAT + amp * np.tile(row, (ny, 1))


def test_theta_half_second_order_for_hyperdiffusion(orc):
    """A y-invariant field about C0 = 1/sqrt(3): the mixed term vanishes
    exactly, the linearised dynamics is pure hyper-diffusion, and the
    Crank-Nicolson variant converges at second order in dt (error ratios 4
    under halving); theta = 1 at first order (ratios 2)."""
    gamma, T = 0.01, 1.0
    C0 = _modes_x(64, 8, (1, 2, 3, 5), 1e-7)
    dts = (0.1, 0.05, 0.025)
    e_half = _order_study(orc, C0, gamma, T, dts, 0.5)
    e_one = _order_study(orc, C0, gamma, T, dts, 1.0)
    r_half = [e_half[0] / e_half[1], e_half[1] / e_half[2]]
    r_one = [e_one[0] / e_one[1], e_one[1] / e_one[2]]
    print("theta 1/2 errors", e_half, r_half, "theta 1 errors", e_one, r_one)
    assert all(3.6 < r < 4.4 for r in r_half), r_half
    assert all(1.8 < r < 2.2 for r in r_one), r_one
    assert e_half[-1] < 0.02 * e_one[-1]


def test_theta_half_first_order_with_mixed_term(orc):
    """A diagonal mode: the explicit mixed term -2 gamma dt D_x D_y C^n makes
    the step first order (error ratios 2), as the paper reports for its scheme
    once terms beyond hyper-diffusion enter."""
    n, gamma, T = 32, 0.01, 1.0
    x = np.arange(n) * TWO_PI / n
    X, Y = np.meshgrid(x, x, indexing="xy")
    C0 = C_FLAT + 1e-7 * (np.cos(2 * X + 2 * Y) + np.cos(3 * X - Y + 1.0))
    e = _order_study(orc, C0, gamma, T, (0.05, 0.025, 0.0125), 0.5)
    r = [e[0] / e[1], e[1] / e[2]]
    print("diagonal modes, theta 1/2 errors", e, r)
    assert all(1.8 < q < 2.3 for q in r), r


def test_theta_half_conservation_and_odd_symmetry(orc):
    C0 = orc.init_field((64, 64), 0.2, 0.1, 9)
    C = orc.step(C0, 0.01, 1e-3, 300, theta=0.5)
    eps = np.finfo(np.float64).eps
    assert abs(orc.mean(C) - orc.mean(C0)) <= 300 * eps
    np.testing.assert_array_equal(orc.step(-C0, 0.01, 1e-3, 50, theta=0.5),
                                  -orc.step(C0, 0.01, 1e-3, 50, theta=0.5))


def _max_growth_at_pure_phase(n, gamma, dt):
    """Largest |G| of the Crank-Nicolson step over all modes, linearised about
    C = 1 (closed form)."""
    best = 0.0
    for kx in range(n // 2 + 1):
        for ky in range(n // 2 + 1):
            best = max(best, abs(refs.amplification((kx, ky), (n, n), TWO_PI, gamma, dt, 1.0, theta=0.5)))
    return best


def test_theta_half_unstable_about_pure_phases_at_large_rho(orc):
    """About a pure phase (C = 1, where 3 C^2 - 1 = 2) the explicit nonlinear
    and mixed terms push diagonal modes of the Crank-Nicolson step past
    |G| = 1 once gamma dt / h^4 exceeds a few hundredths: at 64^2, gamma 0.01,
    dt 1e-3 (rho = 1.7) the worst mode grows by 1.47 per step, and seeded
    noise about C = 1 grows accordingly, while theta = 1 damps it.  At
    dt = 2e-5 (rho = 0.034) the same noise decays."""
    n, gamma = 64, 0.01
    g_big = _max_growth_at_pure_phase(n, gamma, 1e-3)
    g_small = _max_growth_at_pure_phase(n, gamma, 2e-5)
    assert 1.4 < g_big < 1.5 and g_small <= 1.0 + 1e-12, (g_big, g_small)
    noise = orc.init_field((n, n), 0.0, 1e-9, 5)
    for theta, dt, grows in ((0.5, 1e-3, True), (1.0, 1e-3, False), (0.5, 2e-5, False)):
        C = orc.step(1.0 + noise, gamma, dt, 20, theta=theta)
        amp = float(np.abs(C - 1.0).max())
        print(f"theta {theta}, dt {dt}: noise 1e-9 -> {amp:.2e} after 20 steps")
        if grows:
            assert amp > 1e-9 * 1.3**20
        else:
            assert amp < 1e-9
