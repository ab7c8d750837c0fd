"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Bar (FP64): max |C_gpu - C_oracle| <= 1e-10 over the run, and F, dF/dt (both
forms), <C> and beta within 1e-10 relative (absolute where the value is
near zero).  Rounding-order differences between the two implementations
stay at 1e-14..1e-13 over these runs, so the bar leaves a wide margin while
still catching any real discrepancy (a wrong coefficient or index shows at
1e-4 or worse after one step).
"""
import numpy as np
import pytest

import oracle
from paper_1911_03386_amd import CH_F32_BULK, CH_F64, ChError, Ensemble, make_desc
from paper_1911_03386_amd import ch as chmod

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _ref_field(d, shape):
    return oracle.init_field(shape, d.c0, d.noise, d.seed)


def _L(d):
    return [d.L[a] for a in range(d.dim)]


def _check_series(ser, S, tol=TOL):
    assert ser.shape == S.shape, (ser.shape, S.shape)
    np.testing.assert_array_equal(ser[:, 0], S[:, 0])
    for col in (1, 2, 3, 5):
        ref = S[:, col]
        scale = max(np.abs(ref).max(), 1e-300)
        err = np.abs(ser[:, col] - ref).max() / scale
        assert err <= tol, (col, err)
    # beta: relative to its scale, absolute where it is ~0
    err = np.abs(ser[:, 4] - S[:, 4]).max()
    assert err <= tol * max(1.0, np.abs(S[:, 4]).max()), err


def test_c1_parity_2000_steps():
    """128^2, gamma = 0.01, dt = 1e-3, 2000 steps, FP64, samples every 10 steps."""
    gamma, dt, N, K = 0.01, 1e-3, 2000, 10
    d = make_desc((128, 128), gamma, dt, c0=0.0, noise=0.1, seed=1)
    ens = Ensemble([d], prec=CH_F64, cadence=K, max_samples=N // K + 1)
    ens.init_random()
    C = _ref_field(d, (128, 128))
    np.testing.assert_array_equal(ens.get_field(0), C)
    worst = 0.0
    for seg in range(4):
        ens.step(N // 4)
        C = oracle.step(C, gamma, dt, N // 4)
        worst = max(worst, float(np.abs(ens.get_field(0) - C).max()))
    print(f"c1 max |C - oracle| over 2000 steps: {worst:.3e}")
    assert worst <= TOL
    _, S = oracle.run_series(_ref_field(d, (128, 128)), gamma, dt, N, K=K)
    _check_series(ens.beta_series(0), S)
    ens.close()


SHAPES = [
    # (n (x, y[, z]), gamma, dt, L, c0)
    ((64, 48), 0.01, 1e-3, None, 0.0),
    ((160, 96), 0.02, 5e-4, (5.0, 3.0), 0.2),       # 10 chunks per x-line, ragged y-bands
    ((40, 24), 0.01, 1e-3, None, 0.1),               # P not a power of two
    ((8, 8), 0.05, 1e-3, (1.0, 1.0), 0.0),           # smallest grid
    ((256, 8), 0.01, 2e-4, None, -0.3),
    ((24, 16, 20), 0.01, 5e-4, None, 0.0),           # 3D
    ((32, 8, 12), 0.02, 1e-3, (3.0, 2.0, 4.0), 0.25),
]


@pytest.mark.parametrize("prec", [CH_F64])
@pytest.mark.parametrize("spec", SHAPES, ids=[str(s[0]) for s in SHAPES])
def test_shapes_parity(spec, prec):
    n, gamma, dt, L, c0 = spec
    d = make_desc(n, gamma, dt, c0=c0, noise=0.1, seed=3, L=L)
    N, K = 60, 7
    ens = Ensemble([d], prec=prec, cadence=K, max_samples=N // K + 1)
    ens.init_random()
    ens.step(N)
    shape = ens.shape(0)
    Cref, S = oracle.run_series(_ref_field(d, shape), gamma, dt, N, K=K, L=_L(d))
    err = float(np.abs(ens.get_field(0) - Cref).max())
    print(f"{n}: max |C - oracle| = {err:.3e}")
    assert err <= TOL
    _check_series(ens.beta_series(0), S)
    ens.close()


def test_mixed_batch_parity():
    """Members of different sizes, dimensions and parameters in one context."""
    descs = [
        make_desc((64, 64), 0.01, 1e-3, c0=0.0, noise=0.1, seed=10),
        make_desc((32, 64), 0.005, 5e-4, c0=0.3, noise=0.05, seed=11, L=(3.0, 6.0)),
        make_desc((64, 64), 0.02, 1e-3, c0=-0.2, noise=0.05, seed=12),
        make_desc((16, 16, 16), 0.01, 5e-4, c0=0.0, noise=0.05, seed=13),
        make_desc((128, 32), 0.01, 2e-3, c0=0.1, noise=0.1, seed=14),
    ]
    N, K = 40, 10
    ens = Ensemble(descs, prec=CH_F64, cadence=K, max_samples=N // K + 1)
    assert ens.num_classes() == 4
    ens.init_random()
    ens.step(N)
    F, mC = ens.energy()
    for m, d in enumerate(descs):
        shape = ens.shape(m)
        Cref, S = oracle.run_series(_ref_field(d, shape), d.gamma, d.dt, N, K=K, L=_L(d))
        err = float(np.abs(ens.get_field(m) - Cref).max())
        assert err <= TOL, (m, err)
        _check_series(ens.beta_series(m), S)
        assert abs(F[m] - S[-1, 1]) <= TOL * S[-1, 1]
        assert abs(mC[m] - S[-1, 5]) <= 1e-14
    ens.close()


def _all_tiles(ens, cls, n, prec):
    """Every tile shape the autotuner may choose for a 2D class."""
    out = []
    nx, ny = n
    for waves in (1, 2, 4):
        for cx, rl in ((4, 1), (8, 1), (16, 1), (32, 1), (64, 1), (4, 2), (8, 2), (16, 2), (32, 2),
                       (4, 4), (8, 4), (16, 4)):
            if nx % cx or nx // cx > 64:
                continue
            for cy in (4, 8, 16, 32) + ((64,) if prec == CH_F32_BULK else ()):
                if ny % cy:
                    continue
                P = ny // cy
                for b in (1, 2, 4, 8, 16, 32, 64):
                    if nx % b == 0 and b * P <= 512:
                        for units in (1, 2, 3):
                            out.append((cx, rl, waves, units, cy, b))
    return out


def test_split_classes_on_streams_parity():
    """16 members of one shape: the class is split into 4 classes of 4 that run
    on 4 streams.  Every member against the oracle; graph replays, direct
    launches and a different graph length give bitwise equal results."""
    descs = [make_desc((64, 32), 0.01, 1e-3, c0=0.05 * (m % 5) - 0.1, noise=0.1, seed=300 + m)
             for m in range(16)]
    N, K = 30, 10
    runs = []
    for gsteps in (16, 0, 7):
        ens = Ensemble(descs, prec=CH_F64, cadence=K, max_samples=N // K + 1)
        assert ens.num_classes() == 4
        ens.set_graph_steps(gsteps)
        ens.init_random()
        ens.step(N)
        runs.append((np.stack([ens.get_field(m) for m in range(16)]),
                     np.stack([ens.beta_series(m) for m in range(16)])))
        ens.close()
    for C, S in runs[1:]:
        np.testing.assert_array_equal(C, runs[0][0])
        np.testing.assert_array_equal(S, runs[0][1])
    for m in (0, 3, 4, 9, 15):
        d = descs[m]
        Cref, S = oracle.run_series(_ref_field(d, (32, 64)), d.gamma, d.dt, N, K=K)
        err = float(np.abs(runs[0][0][m] - Cref).max())
        assert err <= TOL, (m, err)
        _check_series(runs[0][1][m], S)


def test_every_tile_shape_parity_2d():
    n, gamma, dt = (128, 64), 0.01, 1e-3
    d = make_desc(n, gamma, dt, c0=0.1, noise=0.1, seed=21)
    N = 12
    Cref = oracle.step(_ref_field(d, (64, 128)), gamma, dt, N)
    ens = Ensemble([d], prec=CH_F64, cadence=5, max_samples=N // 5 + 1)
    _, S = oracle.run_series(_ref_field(d, (64, 128)), gamma, dt, N, K=5)
    tried = 0
    seen_units = set()
    for cx, rl, waves, units, cy, b in _all_tiles(ens, 0, n, CH_F64):
        try:
            ens.set_tiles(0, cx, rl, waves, units, cy, b)
        except ChError:
            continue
        ens.init_random()
        ens.step(N)
        err = float(np.abs(ens.get_field(0) - Cref).max())
        assert err <= TOL, ((cx, rl, waves, units, cy, b), err)
        _check_series(ens.beta_series(0), S)
        tried += 1
        seen_units.add(units)
    assert tried >= 80 and seen_units == {1, 2, 3}
    ens.close()


def test_every_tile_shape_parity_3d():
    n, gamma, dt = (32, 16, 24), 0.01, 5e-4
    d = make_desc(n, gamma, dt, c0=0.0, noise=0.1, seed=22)
    N = 6
    Cref = oracle.step(_ref_field(d, (24, 16, 32)), gamma, dt, N)
    _, S = oracle.run_series(_ref_field(d, (24, 16, 32)), gamma, dt, N, K=5)
    ens = Ensemble([d], prec=CH_F64, cadence=5, max_samples=N // 5 + 1)
    tried = 0
    seen_units = set()
    for cx, rl in ((4, 1), (8, 1), (16, 1), (32, 1), (4, 2), (8, 2), (16, 2), (4, 4), (8, 4)):
        for waves in (1, 4):
            for units in (1, 3, 8, 24):
                for cy, by in ((4, 8), (8, 32), (16, 2)):
                    for cz, bz in ((4, 32), (8, 16), (24 // 4, 1), (8, 64)):
                        if 24 % cz:
                            continue
                        try:
                            ens.set_tiles(0, cx, rl, waves, units, cy, by, cz, bz)
                        except ChError:
                            continue
                        ens.init_random()
                        ens.step(N)
                        err = float(np.abs(ens.get_field(0) - Cref).max())
                        assert err <= TOL, ((cx, rl, waves, units, cy, by, cz, bz), err)
                        _check_series(ens.beta_series(0), S)
                        tried += 1
                        seen_units.add(units)
    assert tried >= 40 and seen_units == {1, 3, 8, 24}
    ens.close()


def test_several_bands_fp32_2d_ragged():
    """FP32 bulk, 2D, several y-bands per block, with a ragged last band (72
    lines in bands of 16 or 32) and a ragged last group of bands, against the
    oracle from the same FP32-rounded field; sample steps included."""
    n, gamma, dt = (256, 72), 0.01, 1e-3
    d = make_desc(n, gamma, dt, c0=-0.1, noise=0.1, seed=24)
    N = 12
    C0 = _ref_field(d, (72, 256)).astype(np.float32).astype(np.float64)
    Cref = oracle.step(C0, gamma, dt, N)
    ens = Ensemble([d], prec=CH_F32_BULK, cadence=5, max_samples=N // 5 + 1)
    tried = 0
    for cx, rl in ((4, 1), (8, 1), (16, 1), (32, 1), (8, 2), (16, 2)):
        for waves in (2, 4):
            for units in (2, 3):
                try:
                    ens.set_tiles(0, cx, rl, waves, units, 8, 8)
                except ChError:
                    continue
                ens.init_random()
                ens.step(N)
                err = float(np.abs(ens.get_field(0) - Cref).max())
                assert err <= 2e-5, ((cx, rl, waves, units), err)
                tried += 1
    assert tried >= 12
    ens.close()


def test_plane_ring_fp32_3d():
    """FP32 bulk, 3D, several z-planes per block (ragged last unit: 20 planes
    in units of 8) against the oracle from the same FP32-rounded field."""
    n, gamma, dt = (64, 24, 20), 0.01, 5e-4
    d = make_desc(n, gamma, dt, c0=0.1, noise=0.1, seed=23)
    N = 6
    C0 = _ref_field(d, (20, 24, 64)).astype(np.float32).astype(np.float64)
    Cref = oracle.step(C0, gamma, dt, N)
    ens = Ensemble([d], prec=CH_F32_BULK, cadence=5, max_samples=N // 5 + 1)
    tried = 0
    for cx, rl in ((4, 1), (8, 1), (16, 1), (32, 1), (4, 2), (8, 2), (16, 2)):
        for waves in (1, 2, 4):
            try:
                ens.set_tiles(0, cx, rl, waves, 8, 8, 8, 4, 16)
            except ChError:
                continue
            ens.init_random()
            ens.step(N)
            err = float(np.abs(ens.get_field(0) - Cref).max())
            assert err <= 2e-5, ((cx, rl, waves), err)
            tried += 1
    assert tried >= 8
    ens.close()


def test_graph_and_eager_bitwise_equal_and_deterministic():
    d = make_desc((128, 128), 0.01, 1e-3, c0=0.0, noise=0.1, seed=5)
    outs = []
    for g in (0, 16, 16, 7):
        ens = Ensemble([d], prec=CH_F64, cadence=10, max_samples=11)
        ens.set_graph_steps(g)
        ens.init_random()
        ens.step(50)
        ens.step(50)
        outs.append((ens.get_field(0), ens.beta_series(0)))
        ens.close()
    for C, S in outs[1:]:
        np.testing.assert_array_equal(C, outs[0][0])
        np.testing.assert_array_equal(S, outs[0][1])


def test_resume_bitwise():
    d = make_desc((64, 64), 0.01, 1e-3, c0=0.0, noise=0.1, seed=6)
    a = Ensemble([d], prec=CH_F64, cadence=10, max_samples=21)
    a.init_random()
    a.step(200)
    full = a.get_field(0)
    sa = a.beta_series(0)
    b = Ensemble([d], prec=CH_F64, cadence=10, max_samples=21)
    b.init_random()
    b.step(100)
    mid = b.get_field(0)
    b.close()
    c = Ensemble([d], prec=CH_F64, cadence=10, max_samples=21)
    c.set_field(0, mid)
    c.set_step(100)
    assert c.step_count == 100
    c.step(100)
    np.testing.assert_array_equal(c.get_field(0), full)
    sc = c.beta_series(0)
    # samples after the restore point match exactly; the restore sample itself
    # is one-sided
    np.testing.assert_array_equal(sc[11:], sa[11:])
    assert np.all(np.isnan(sc[:10, 1]))
    a.close()
    c.close()


def test_energy_and_set_field_parity():
    rng = np.random.default_rng(0)
    d = make_desc((48, 32), 0.02, 1e-3)
    ens = Ensemble([d], prec=CH_F64, cadence=10, max_samples=2)
    C = 0.3 * rng.standard_normal((32, 48))
    ens.set_field(0, C)
    F, mC = ens.energy()
    assert abs(F[0] - oracle.energy(C, 0.02)) <= 1e-13 * F[0]
    assert abs(mC[0] - oracle.mean(C)) <= 1e-15
    ens.close()


def test_nonfinite_flag():
    d = make_desc((32, 32), 0.01, 1e-3, c0=0.0, noise=0.1, seed=2)
    ens = Ensemble([d], prec=CH_F64, cadence=1, max_samples=11)
    big = np.full((32, 32), 60.0)
    big[3, 4] = -60.0
    ens.set_field(0, big)
    ens.step(10)
    with pytest.raises(ChError) as e:
        ens.energy()
    assert e.value.status == chmod.CH_ENONFINITE
    with pytest.raises(ChError) as e:
        ens.beta_series(0)
    assert e.value.status == chmod.CH_ENONFINITE
    ens.close()


def test_sample_capacity_and_destroyed_context():
    d = make_desc((32, 32), 0.01, 1e-3)
    ens = Ensemble([d], prec=CH_F64, cadence=10, max_samples=3)
    ens.step(29)
    with pytest.raises(ChError) as e:
        ens.step(1)
    assert e.value.status == chmod.CH_ESTATE
    ctx = ens.ctx
    ens.close()
    assert chmod.load().ch_step(ctx, 1) == chmod.CH_ESTATE


def test_fp32_trajectory_error_short_window():
    """FP32 bulk against the FP64 oracle from the same (rounded) initial field."""
    gamma, dt, N, K = 0.01, 1e-3, 200, 10
    d = make_desc((128, 128), gamma, dt, c0=0.0, noise=0.1, seed=1)
    ens = Ensemble([d], prec=CH_F32_BULK, cadence=K, max_samples=N // K + 1)
    ens.init_random()
    C0 = ens.get_field(0)  # FP32-rounded initial condition, widened
    ref0 = _ref_field(d, (128, 128))
    assert np.abs(C0 - ref0).max() <= 6e-8 * 0.1 + 1e-12
    ens.step(N)
    Cref, S = oracle.run_series(C0, gamma, dt, N, K=K)
    err = float(np.abs(ens.get_field(0) - Cref).max())
    ser = ens.beta_series(0)
    ferr = float(np.abs(ser[:, 1] - S[:, 1]).max() / S[:, 1].max())
    drift = float(np.abs(ser[:, 5] - ser[0, 5]).max())
    print(f"FP32 128^2 x 200 steps: max|dC| = {err:.2e}, max rel dF = {ferr:.2e}, <C> drift = {drift:.2e}")
    assert err < 1e-4
    assert ferr < 1e-5
    assert drift < 1e-6


def test_autotune_keeps_parity_and_caches(tmp_path):
    descs = [make_desc((64, 32), 0.01, 1e-3, c0=0.0, noise=0.1, seed=31),
             make_desc((16, 16, 8), 0.01, 5e-4, c0=0.2, noise=0.05, seed=32)]
    cache = str(tmp_path / "tune.txt")
    N = 20
    ens = Ensemble(descs, prec=CH_F64, cadence=10, max_samples=N // 10 + 1)
    ens.init_random()
    ens.autotune(cache)
    text = open(cache).read()
    assert text.count("\n") == 2 and ":f64:2D:64x32x1:m1 " in text
    plan = ens.describe()
    ens.step(N)
    for m, d in enumerate(descs):
        shape = ens.shape(m)
        ref = oracle.step(_ref_field(d, shape), d.gamma, d.dt, N, L=_L(d))
        assert float(np.abs(ens.get_field(m) - ref).max()) <= TOL
    ens.close()
    # a second context takes the cached shapes without timing again
    ens2 = Ensemble(descs, prec=CH_F64, cadence=10, max_samples=N // 10 + 1)
    ens2.autotune(cache)
    assert ens2.describe() == plan
    ms = ens2.time_kernels(3)
    assert ms[0] > 0 and ms[1] > 0 and ms[2] > 0
    assert ens2.step_count == 3
    ens2.close()


def test_autotune_split_classes(tmp_path):
    """8 members of one shape form 2 classes of 4 with one cache key; the joint
    stage of the tuner times them together.  Parity afterwards."""
    descs = [make_desc((64, 32), 0.01, 1e-3, c0=0.1, noise=0.1, seed=400 + m) for m in range(8)]
    cache = str(tmp_path / "tune.txt")
    N = 20
    ens = Ensemble(descs, prec=CH_F64, cadence=10, max_samples=N // 10 + 1)
    assert ens.num_classes() == 2
    ens.autotune(cache)
    text = open(cache).read()
    assert text.count("\n") == 1 and ":f64:2D:64x32x1:m4 " in text
    ens.init_random()
    ens.step(N)
    for m in (0, 5, 7):
        d = descs[m]
        ref = oracle.step(_ref_field(d, (32, 64)), d.gamma, d.dt, N)
        assert float(np.abs(ens.get_field(m) - ref).max()) <= TOL
    ens.close()


def test_caller_captured_graph_replays():
    """The caller captures ch_step on the context's stream in a graph of its
    own (the library then launches directly, forking its class streams into
    the capture) and replays it several times, with its own eager work and
    synchronisations between the replays.  Every replay equals the same steps
    taken eagerly."""
    import torch

    descs = [make_desc((64, 32), 0.01, 1e-3, c0=0.05 * (m % 3), noise=0.1, seed=600 + m)
             for m in range(16)]  # 4 classes on 4 streams
    chunk, nrep, K = 20, 3, 10
    ref = Ensemble(descs, prec=CH_F64, cadence=K, max_samples=chunk * (nrep + 1) // K + 1)
    ref.set_graph_steps(0)
    ref.init_random()
    ens = Ensemble(descs, prec=CH_F64, cadence=K, max_samples=chunk * (nrep + 1) // K + 1)
    assert ens.num_classes() == 4
    ens.init_random()
    ens.step(chunk)  # warm-up outside the capture (also builds nothing captured)
    ref.step(chunk)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=ens.stream):
        ens.step(chunk)
    scratch = torch.zeros(1 << 20, device="cuda")
    for r in range(nrep):
        g.replay()
        scratch.add_(1.0)  # unrelated eager work between replays
        torch.cuda.synchronize()
        ref.step(chunk)
        for m in (0, 5, 10, 15):
            np.testing.assert_array_equal(ens.get_field(m), ref.get_field(m))
    # the replays advanced the device step counter; the host learns it here
    assert ens.step_count == 2 * chunk
    assert ens.sync_step() == chunk * (nrep + 1) == ens.step_count
    for m in (0, 15):
        np.testing.assert_array_equal(ens.beta_series(m), ref.beta_series(m))
    ens.close()
    ref.close()


@pytest.mark.parametrize("prec", [CH_F64, CH_F32_BULK], ids=["f64", "f32"])
def test_reduction_accuracy_on_identical_fields(prec):
    """F, <C> and the identity term at t = 0 are sums over the same field on
    both sides (the FP32-bulk field rounded to FP32 for the oracle), so their
    difference is the reductions' rounding alone: the oracle's sums are exactly
    rounded, the library's two-level ones stay within 1e-13 of them."""
    d = make_desc((512, 512), 0.01, 1e-3, c0=0.1, noise=0.3, seed=21)
    ens = Ensemble([d], prec=prec, cadence=10, max_samples=2)
    ens.init_random()
    ens.step(10)
    row = ens.beta_series(0)[0]
    ens.close()
    C0 = oracle.init_field((512, 512), d.c0, d.noise, d.seed)
    if prec == CH_F32_BULK:
        C0 = C0.astype(np.float32).astype(np.float64)
    _, S = oracle.run_series(C0, d.gamma, d.dt, 10, K=10)
    errs = {name: abs(row[c] - S[0, c]) / abs(S[0, c]) for name, c in (("F", 1), ("<C>", 5), ("G_id", 3))}
    print("relative differences at t = 0:", {k: f"{v:.2e}" for k, v in errs.items()})
    assert max(errs.values()) <= 1e-13, errs
