"""GPU parity of the Crank-Nicolson ADI variant (theta = 1/2, 2D) against the
oracle's theta-weighted step, through the C ABI.  Same bars as the implicit
scheme: FP64 fields within 1e-10 of the oracle, F, dF/dt (both forms), <C>
and beta within 1e-10 relative; FP32 bulk within 2e-5 over a few steps."""
import numpy as np
import pytest

import oracle
from paper_1911_03386_amd import CH_F32_BULK, CH_F64, ChError, Ensemble, make_desc
from paper_1911_03386_amd import ch as chmod
from tests.test_gpu_parity import TOL, _check_series, _L, _ref_field

pytestmark = pytest.mark.gpu

SHAPES = [
    ((128, 128), 0.01, 1e-3, None, 0.0),
    ((64, 48), 0.02, 5e-4, (3.0, 2.0), 0.2),
    ((160, 96), 0.02, 5e-4, (5.0, 3.0), 0.2),   # 10 chunks per x-line, ragged y-bands
    ((40, 24), 0.01, 1e-3, None, 0.1),
    ((8, 8), 0.05, 1e-3, (1.0, 1.0), 0.0),       # smallest grid: the y halos wrap
    ((256, 8), 0.01, 2e-4, None, -0.3),
]


@pytest.mark.parametrize("spec", SHAPES, ids=[str(s[0]) for s in SHAPES])
def test_cn_shapes_parity(spec):
    n, gamma, dt, L, c0 = spec
    d = make_desc(n, gamma, dt, c0=c0, noise=0.1, seed=41, L=L)
    N, K = 60, 7
    ens = Ensemble([d], prec=CH_F64, cadence=K, max_samples=N // K + 1)
    ens.set_theta(0.5)
    ens.init_random()
    ens.step(N)
    shape = ens.shape(0)
    Cref, S = oracle.run_series(_ref_field(d, shape), gamma, dt, N, K=K, L=_L(d), theta=0.5)
    err = float(np.abs(ens.get_field(0) - Cref).max())
    print(f"CN {n}: max |C - oracle| = {err:.3e} ({ens.describe().strip()})")
    assert err <= TOL
    _check_series(ens.beta_series(0), S)
    ens.close()


def test_cn_128_2000_steps():
    """The 128^2 single grid (gamma 0.01) over 2000 steps, at dt = 2e-5: a
    step where the variant is stable also once the phases separate
    (gamma dt / h^4 = 0.034; at dt = 1e-3 its diagonal modes about C = +-1
    grow by 1.47 per step, see the oracle pins)."""
    gamma, dt, N, K = 0.01, 2e-5, 2000, 10
    d = make_desc((128, 128), gamma, dt, c0=0.0, noise=0.1, seed=1)
    ens = Ensemble([d], prec=CH_F64, cadence=K, max_samples=N // K + 1)
    ens.set_theta(0.5)
    ens.init_random()
    ens.step(N)
    Cref, S = oracle.run_series(_ref_field(d, (128, 128)), gamma, dt, N, K=K, theta=0.5)
    err = float(np.abs(ens.get_field(0) - Cref).max())
    print(f"CN 128^2 max |C - oracle| after 2000 steps: {err:.3e}")
    assert np.all(np.isfinite(Cref)) and err <= TOL
    _check_series(ens.beta_series(0), S)
    ens.close()


def test_cn_every_tile_shape():
    n, gamma, dt = (128, 64), 0.01, 1e-3
    d = make_desc(n, gamma, dt, c0=0.1, noise=0.1, seed=42)
    N = 12
    Cref, S = oracle.run_series(_ref_field(d, (64, 128)), gamma, dt, N, K=5, theta=0.5)
    ens = Ensemble([d], prec=CH_F64, cadence=5, max_samples=N // 5 + 1)
    ens.set_theta(0.5)
    tried = 0
    for cx in (4, 8, 16, 32, 64):
        for waves in (1, 2, 4):
            for cy, b in ((8, 8), (16, 32), (32, 4)):
                try:
                    ens.set_tiles(0, cx, 1, waves, 1, cy, b)
                except ChError:
                    continue
                ens.init_random()
                ens.step(N)
                err = float(np.abs(ens.get_field(0) - Cref).max())
                assert err <= TOL, ((cx, waves, cy, b), err)
                _check_series(ens.beta_series(0), S)
                tried += 1
    # the implicit scheme's shapes that the variant lacks are refused
    for cx, rl, units in ((16, 2, 1), (16, 1, 2)):
        with pytest.raises(ChError):
            ens.set_tiles(0, cx, rl, 4, units, 8, 8)
    assert tried >= 30
    ens.close()


def test_cn_fp32_and_mixed_batch():
    """FP32 bulk (from the same FP32-rounded field) and a batch of several
    shapes and parameters split over classes."""
    descs = [make_desc((256, 72), 0.01, 1e-3, c0=-0.1, noise=0.1, seed=43),
             make_desc((64, 64), 0.005, 5e-4, c0=0.3, noise=0.05, seed=44, L=(3.0, 6.0)),
             make_desc((256, 72), 0.02, 1e-3, c0=0.0, noise=0.1, seed=45)]
    N = 12
    ens = Ensemble(descs, prec=CH_F32_BULK, cadence=5, max_samples=N // 5 + 1)
    ens.set_theta(0.5)
    ens.init_random()
    ens.step(N)
    for m, d in enumerate(descs):
        shape = ens.shape(m)
        C0 = _ref_field(d, shape).astype(np.float32).astype(np.float64)
        Cref = oracle.step(C0, d.gamma, d.dt, N, L=_L(d), theta=0.5)
        err = float(np.abs(ens.get_field(m) - Cref).max())
        print(f"CN FP32 member {m}: max |C - oracle| = {err:.3e}")
        assert err <= 2e-5, (m, err)
    ens.close()


def test_cn_switch_midrun_graphs_and_errors():
    """theta changes from the next step: 30 implicit steps, then 30 CN steps
    (as graph replays and as direct launches, bitwise equal), against the
    oracle doing the same; 3D members and other thetas are refused."""
    d = make_desc((64, 64), 0.01, 1e-3, c0=0.0, noise=0.1, seed=46)
    runs = []
    for g in (16, 0):
        ens = Ensemble([d], prec=CH_F64, cadence=10, max_samples=8)
        ens.set_graph_steps(g)
        ens.init_random()
        ens.step(30)
        ens.set_theta(0.5)
        ens.step(30)
        runs.append((ens.get_field(0), ens.beta_series(0)))
        with pytest.raises(ChError) as e:
            ens.set_theta(0.75)
        assert e.value.status == chmod.CH_EINVAL
        ens.close()
    np.testing.assert_array_equal(runs[0][0], runs[1][0])
    np.testing.assert_array_equal(runs[0][1], runs[1][1])
    C = oracle.step(_ref_field(d, (64, 64)), 0.01, 1e-3, 30)
    C = oracle.step(C, 0.01, 1e-3, 30, theta=0.5)
    assert np.abs(runs[0][0] - C).max() <= TOL
    e3 = Ensemble([make_desc((16, 16, 16), 0.01, 5e-4)], prec=CH_F64, cadence=10, max_samples=2)
    with pytest.raises(ChError) as e:
        e3.set_theta(0.5)
    assert e.value.status == chmod.CH_EUNSUPPORTED
    e3.close()
