"""Device-side ensemble statistics of beta against the oracle's statistics of
the oracle's own beta series (eq. (mup), eq. (beta0_stats), the fit
mu_2 = k t, histograms).  FP64 members, so the two beta series agree to
about 1e-11 relative; the statistics are compared at 1e-9."""
import math

import numpy as np
import pytest

import oracle
from oracle import stats as ostats
from paper_1911_03386_amd import CH_F64, ChError, Ensemble, make_desc

pytestmark = pytest.mark.gpu

M, N, K = 12, 2000, 10
SHAPE = (32, 32)


def _descs():
    return [make_desc(SHAPE, 0.01, 1e-3, c0=(0.0 if m < M // 2 else 0.3), noise=0.1, seed=500 + m)
            for m in range(M)]


@pytest.fixture(scope="module")
def runs():
    descs = _descs()
    ens = Ensemble(descs, prec=CH_F64, cadence=K, max_samples=N // K + 1)
    ens.init_random()
    ens.step(N)
    series = []
    for d in descs:
        _, S = oracle.run_series(oracle.init_field(SHAPE[::-1], d.c0, d.noise, d.seed), d.gamma, d.dt, N, K=K)
        series.append(S)
    t = series[0][:, 0]
    beta = np.stack([S[:, 4] for S in series])  # (M, J)
    yield ens, t, beta
    ens.close()


def _close(a, b, rel):
    scale = max(float(np.nanmax(np.abs(b))), 1e-300)
    return float(np.nanmax(np.abs(np.asarray(a) - np.asarray(b)))) <= rel * scale + 1e-15


def test_moments_vs_oracle(runs):
    ens, t, beta = runs
    tg, mu = ens.ensemble_moments(pmax=4)
    np.testing.assert_array_equal(tg, t)
    ref = ostats.ensemble_moments(beta, 4)
    for p in range(4):
        assert _close(mu[:, p], ref[:, p], 1e-9), p
    # a subset of members
    sel = [0, 3, 7, 11]
    _, mus = ens.ensemble_moments(members=sel, pmax=3)
    refs = ostats.ensemble_moments(beta[sel], 3)
    for p in range(3):
        assert _close(mus[:, p], refs[:, p], 1e-9), p


def test_window_vs_oracle(runs):
    ens, t, beta = runs
    ref = ostats.ensemble_moments(beta, 2)
    for t1, t2 in ((0.5, 2.0), (1.0, 1.5), (0.0, 2.0)):
        b0, k = ens.ensemble_window(t1, t2)
        rb0, rk = ostats.ensemble_window(t, ref[:, 0], ref[:, 1], t1, t2)
        assert math.isclose(b0, rb0, rel_tol=1e-9), (t1, t2, b0, rb0)
        assert math.isclose(k, rk, rel_tol=1e-9), (t1, t2, k, rk)
    half = list(range(M // 2))
    b0, k = ens.ensemble_window(1.0, 2.0, members=half)
    refh = ostats.ensemble_moments(beta[half], 2)
    rb0, rk = ostats.ensemble_window(t, refh[:, 0], refh[:, 1], 1.0, 2.0)
    assert math.isclose(b0, rb0, rel_tol=1e-9) and math.isclose(k, rk, rel_tol=1e-9)
    # a window without samples
    b0, k = ens.ensemble_window(1.0001, 1.0005)
    assert math.isnan(b0) and math.isnan(k)


def test_histogram_vs_oracle(runs):
    ens, t, beta = runs
    lo, hi, nb = 0.0, 0.6, 12
    got = ens.beta_histogram(1.0, 2.0, lo, hi, nb).astype(np.int64)
    ref = ostats.beta_histogram(beta, t, 1.0, 2.0, lo, hi, nb)
    assert got.sum() == ref.sum()
    # only values within the series' agreement of a bin edge may change bins
    w = beta[:, [j for j in range(len(t)) if 1.0 <= t[j] <= 2.0]].ravel()
    edges = lo + (hi - lo) * np.arange(nb + 1) / nb
    near = int(sum(np.any(np.abs(v - edges) <= 1e-9 * max(abs(v), 1.0)) for v in w))
    assert int(np.abs(got - ref).sum()) <= 2 * near, (got, ref, near)


def test_statistics_errors(runs):
    ens, _, _ = runs
    with pytest.raises(ChError):
        ens.ensemble_moments(pmax=9)
    with pytest.raises(ChError):
        ens.ensemble_moments(members=[0, M])
    with pytest.raises(ChError):
        ens.beta_histogram(0.0, 1.0, 0.0, 1.0, 0)
    with pytest.raises(ChError):
        ens.beta_histogram(0.0, 1.0, 1.0, 0.0, 4)
    with pytest.raises(ChError):
        ens.ensemble_window(2.0, 1.0)
    # a selection longer than the ensemble is refused before anything runs;
    # one of the ensemble's own size may repeat members (a bootstrap resample)
    with pytest.raises(ChError) as e:
        ens.ensemble_moments(members=[0] * (M + 1), pmax=2)
    assert "nm" in str(e.value)
    for call in (lambda: ens.ensemble_window(0.0, 2.0, members=list(range(M)) + [0]),
                 lambda: ens.beta_histogram(0.0, 2.0, 0.0, 1.0, 4, members=[1] * (M + 1))):
        with pytest.raises(ChError):
            call()
    boot = [3] * M
    _, mub = ens.ensemble_moments(members=boot, pmax=2)
    _, mu3 = ens.ensemble_moments(members=[3], pmax=2)
    np.testing.assert_allclose(mub[:, 0], mu3[:, 0], rtol=1e-14, atol=1e-16)
    mixed = Ensemble([make_desc(SHAPE, 0.01, 1e-3, seed=1), make_desc(SHAPE, 0.01, 5e-4, seed=2)],
                     prec=CH_F64, cadence=K, max_samples=3)
    mixed.init_random()
    with pytest.raises(ChError):
        mixed.ensemble_moments()
    t, mu = mixed.ensemble_moments(members=[1], pmax=2)  # one dt: fine
    assert len(t) == 1 and mu[0, 0] == 0.0 and mu[0, 1] == 0.0
    mixed.close()
