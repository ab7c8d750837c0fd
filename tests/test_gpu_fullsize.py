"""Full-size checks in the benchmark's launch configuration.

* the first steps of every benchmark workload against the oracle, element by
  element, for the members the oracle can afford;
* properties that hold at any size over whole runs: conservation of <C>,
  monotone F;
* the FP32-bulk ensemble against the FP64 ensemble from the same initial
  conditions: the paired ensemble-mean beta difference over the second half of
  the run (bar: 1e-3).
"""
import numpy as np
import pytest

import oracle
from paper_1911_03386_amd import CH_F32_BULK, CH_F64, Ensemble, workloads

pytestmark = pytest.mark.gpu


def _shape(d):
    return tuple(d.n[a] for a in range(d.dim))[::-1]


def _ens(wl, prec=None, max_samples=None):
    ms = max_samples if max_samples is not None else wl.steps // wl.cadence + 1
    return Ensemble(wl.descs, prec=wl.prec if prec is None else prec, cadence=wl.cadence,
                    max_samples=ms)


def _first_steps_vs_oracle(wl, members, nsteps, tol):
    ens = _ens(wl, max_samples=nsteps // wl.cadence + 2)
    ens.init_random()
    ens.step(nsteps)
    for m in members:
        d = wl.descs[m]
        C0 = oracle.init_field(_shape(d), d.c0, d.noise, d.seed)
        if wl.prec == CH_F32_BULK:
            C0 = C0.astype(np.float32).astype(np.float64)
        ref = oracle.step(C0, d.gamma, d.dt, nsteps, L=[d.L[a] for a in range(d.dim)])
        err = float(np.abs(ens.get_field(m) - ref).max())
        print(f"{wl.name} member {m}: {nsteps} steps, max |C - oracle| = {err:.3e}")
        assert err <= tol, (m, err)
    ens.close()


def test_c2_first_steps_parity():
    _first_steps_vs_oracle(workloads.c2(), [0], 20, 1e-12)


def test_c3_fp64_first_steps_parity():
    _first_steps_vs_oracle(workloads.c3(CH_F64), [0, 31, 32, 63], 20, 1e-12)


def test_c3_fp32_first_steps_close():
    _first_steps_vs_oracle(workloads.c3(CH_F32_BULK), [0, 63], 20, 2e-5)


def test_c4_first_steps_close():
    wl = workloads.c4()
    _first_steps_vs_oracle(wl, [0, 31, 32, 48, 51], 10, 2e-5)


def test_c5_first_step_close():
    _first_steps_vs_oracle(workloads.c5(), [0, 7], 2, 2e-5)


def test_c2_full_run_invariants():
    wl = workloads.c2()
    ens = _ens(wl)
    ens.init_random()
    ens.step(wl.steps)
    S = ens.beta_series(0)
    assert S.shape[0] == wl.steps // wl.cadence + 1
    assert np.all(np.isfinite(S[:, 1]))
    assert np.abs(S[:, 5] - S[0, 5]).max() <= 1e-13
    assert np.all(np.diff(S[:, 1]) <= 1e-12 * S[:-1, 1])
    ens.close()


def _window_stats(b64, b32, t):
    """Paired ensemble-mean difference of beta over t in [t_N/2, t_N]."""
    W = t >= t[-1] / 2
    diff = (b32 - b64)[:, W]            # members x samples
    mean_t = diff.mean(axis=0)           # ensemble mean at each sample
    return float(mean_t.mean()), float(np.abs(mean_t).max()), float(diff.mean(axis=1).std(ddof=1) / np.sqrt(diff.shape[0]))


def test_c3_fp32_vs_fp64_ensemble_mean_beta():
    runs = {}
    for prec in (CH_F64, CH_F32_BULK):
        wl = workloads.c3(prec)
        ens = _ens(wl)
        ens.init_random()
        ens.step(wl.steps)
        runs[prec] = np.stack([ens.beta_series(m) for m in range(len(wl.descs))])
        ens.close()
    s64, s32 = runs[CH_F64], runs[CH_F32_BULK]
    t = s64[0, :, 0]
    np.testing.assert_array_equal(t, s32[0, :, 0])
    # FP64 run: conservation and monotone energy in every member
    assert np.abs(s64[:, :, 5] - s64[:, :1, 5]).max() <= 1e-13
    assert np.all(np.diff(s64[:, :, 1], axis=1) <= 1e-12 * s64[:, :-1, 1])
    b64, b32 = s64[:, :, 4], s32[:, :, 4]
    d_all, dmax, se = _window_stats(b64, b32, t)
    d_sym, _, _ = _window_stats(b64[:32], b32[:32], t)
    d_asym, _, _ = _window_stats(b64[32:], b32[32:], t)
    W = t >= t[-1] / 2
    print(f"paired window-mean dbeta: all {d_all:.2e} (se {se:.1e}), C0=0 {d_sym:.2e}, C0=0.3 {d_asym:.2e}; "
          f"max_t |ensemble-mean dbeta| {dmax:.2e}; beta64 window mean {b64[:, W].mean():.4f}; "
          f"FP32 <C> drift {np.abs(s32[:, :, 5] - s32[:, :1, 5]).max():.1e}")
    assert abs(d_all) <= 1e-3
    assert abs(d_sym) <= 1e-3 and abs(d_asym) <= 1e-3
