"""Long lines against the FP64 oracle: x-lines of 128 or 256 chunks held by
2 or 4 wavefronts (the chunk scans combined across wavefronts through LDS),
the split form (an RHS tile pass, then the x-solve in place), column sweeps
of up to 256 chunks, and the n = 8192 grids they open (2D).

Bar as in the other parity tests: FP64 fields within 1e-10 of the oracle and
the F, dF/dt, <C>, beta series within 1e-10 relative; FP32-bulk fields within
3e-5 after 20 steps from the FP32-rounded initial field.
"""
import numpy as np
import pytest

import oracle
from paper_1911_03386_amd import CH_F32_BULK, CH_F64, ChError, Ensemble, make_desc

from tests.test_gpu_parity import TOL, _check_series

pytestmark = pytest.mark.gpu


def _col_shape(ny, prec):
    """A y-sweep shape valid for ny: chunk length and columns per block."""
    for cy in (4, 8, 16, 32):
        if ny % cy == 0 and ny // cy <= 256:
            return cy, max(1, min(16, 512 // (ny // cy)))
    raise ValueError(ny)


H = 2 * np.pi / 512  # grid spacing of every case (that of the benchmark grids)


def _run(n, prec, tiles=None, N=30, K=7, seed=5, gamma=0.01, dt=5e-4, c0=0.1):
    d = make_desc(n, gamma, dt, c0=c0, noise=0.1, seed=seed, L=(n[0] * H, n[1] * H))
    ens = Ensemble([d], prec=prec, cadence=K, max_samples=N // K + 1)
    if tiles is not None:
        cx, units = tiles
        cy, by = _col_shape(n[1], prec)
        ens.set_tiles(0, cx, 1, 4, units, cy, by, 0, 0)
    plan = ens.describe().strip()
    print("plan:", plan)
    ens.init_random()
    ens.step(N)
    out = (ens.get_field(0), ens.beta_series(0), plan)
    ens.close()
    return d, out


def _oracle(d, N, K, f32=False):
    shape = (d.n[1], d.n[0])
    C0 = oracle.init_field(shape, d.c0, d.noise, d.seed)
    if f32:
        C0 = C0.astype(np.float32).astype(np.float64)
        return oracle.step(C0, d.gamma, d.dt, N, L=[d.L[0], d.L[1]]), None
    return oracle.run_series(C0, d.gamma, d.dt, N, K=K, L=[d.L[0], d.L[1]])


# (nx, ny, chunk length, form): 64 * wavefronts * chunk = nx
WIDE = [
    (1024, 12, 4, "wide"),     # 4 wavefronts per line, 1 line per block
    (1024, 12, 8, "wide"),     # 2 wavefronts per line, 2 lines per block
    (2048, 8, 8, "wide"),
    (2048, 8, 16, "wide"),
    (4096, 8, 16, "wide"),     # (FP64 rows of 4096 with 2 lines per block exceed LDS)
    (8192, 8, 32, "split"),    # FP64 rows of 8192 exceed LDS: RHS tiles, then the x-solve
    (1024, 12, 4, "split"),
]


@pytest.mark.parametrize("spec", WIDE, ids=[f"{s[0]}x{s[1]}-c{s[2]}-{s[3]}" for s in WIDE])
def test_wide_lines_fp64_parity(spec):
    nx, ny, cx, form = spec
    N, K = 30, 7
    d, (C, ser, plan) = _run((nx, ny), CH_F64, tiles=(cx, 0 if form == "split" else 1), N=N, K=K)
    assert f"P={nx // cx} " in plan and (" split" in plan if form == "split" else " wide" in plan), plan
    Cref, S = _oracle(d, N, K)
    err = float(np.abs(C - Cref).max())
    print(f"{nx}x{ny} cx={cx} {form}: max |C - oracle| = {err:.3e}")
    assert err <= TOL
    _check_series(ser, S)


@pytest.mark.parametrize("spec", [(1024, 12, 4), (2048, 8, 16), (4096, 8, 32), (8192, 8, 32)], ids=str)
def test_wide_lines_fp32_close(spec):
    nx, ny, cx = spec
    N = 20
    d, (C, _, plan) = _run((nx, ny), CH_F32_BULK, tiles=(cx, 1), N=N, K=N + 1)
    assert " wide" in plan, plan
    Cref, _ = _oracle(d, N, None, f32=True)
    err = float(np.abs(C - Cref).max())
    print(f"FP32 {nx}x{ny} cx={cx}: max |C - oracle| = {err:.3e}")
    assert err <= 3e-5


def test_default_plans_of_8192_lines():
    """Without tuning: FP64 8192-point x-lines take the split form, FP32 ones
    stage whole rows; both step and match the oracle."""
    for prec, form in ((CH_F64, " split"), (CH_F32_BULK, " wide")):
        d, (C, _, plan) = _run((8192, 8), prec, N=6, K=7)
        assert form in plan, plan
        Cref, _ = _oracle(d, 6, 7, f32=(prec == CH_F32_BULK))
        err = float(np.abs(C - Cref).max())
        print(f"default plan {plan}: max |C - oracle| = {err:.3e}")
        assert err <= (TOL if prec == CH_F64 else 3e-5)


@pytest.mark.parametrize("n,prec", [((8, 8192), CH_F64), ((16, 8192), CH_F32_BULK), ((12, 2048), CH_F64)],
                         ids=["8x8192-f64", "16x8192-f32", "12x2048-f64"])
def test_long_columns_parity(n, prec):
    """y-lines of 128 to 256 chunks (the column sweep's deepest scans)."""
    N, K = 20, 7
    d, (C, ser, plan) = _run(n, prec, N=N, K=K)
    P = int(plan.split("| y cy=")[1].split("P=")[1].split()[0])
    assert P >= 128, plan
    f32 = prec == CH_F32_BULK
    Cref, S = _oracle(d, N, K, f32=f32)
    err = float(np.abs(C - Cref).max())
    print(f"{n} {plan}: max |C - oracle| = {err:.3e}")
    assert err <= (3e-5 if f32 else TOL)
    if not f32:
        _check_series(ser, S)


def test_column_shapes_beyond_the_scan_are_refused():
    """512 chunks per column exceed the column scan: refused, plan unchanged."""
    d = make_desc((64, 2048), 0.01, 1e-3)
    ens = Ensemble([d], prec=CH_F64, cadence=10, max_samples=2)
    before = ens.describe()
    with pytest.raises(ChError):
        ens.set_tiles(0, 16, 1, 4, 1, 4, 1, 0, 0)  # 2048 / 4 = 512 chunks
    assert ens.describe() == before
    ens.close()


def test_single_grid_wide_plans_match_narrow():
    """A 1024^2 FP64 grid with the narrow plan (16 per lane, 64 chunks) and
    with lines of 256 and 128 chunks: the same fields to rounding, and the
    oracle over the first steps."""
    N, K = 10, 5
    fields = {}
    for cx in (16, 4, 8):
        d, (C, ser, plan) = _run((1024, 1024), CH_F64, tiles=(cx, 1), N=N, K=K, dt=1e-3, c0=0.0)
        fields[cx] = (C, ser)
    Cref, S = _oracle(d, N, K)
    for cx, (C, ser) in fields.items():
        err = float(np.abs(C - Cref).max())
        print(f"1024^2 cx={cx}: max |C - oracle| = {err:.3e}")
        assert err <= TOL
        _check_series(ser, S)
