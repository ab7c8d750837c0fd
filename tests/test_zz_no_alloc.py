"""ch_step_static, the allocation-free stepping entry point, against the
context path (ch_create / ch_step / ch_energy) on the same members and
initial fields: two calls in a row, the second on a smaller ensemble, and a
3D FP32 call.  Both paths run the same kernels with the same tile shapes, so
the fields agree to the FP64 parity bar (1e-12 here; they are expected to be
bit-identical) and F, <C> to 1e-12 relative."""
import numpy as np
import pytest
import torch

from paper_1911_03386_amd import ch

pytestmark = pytest.mark.gpu

TOL = {ch.CH_F64: 1e-12, ch.CH_F32_BULK: 1e-6}


def _reference(descs, prec, nsteps):
    """Initial fields, fields after nsteps and (F, <C>) by the context path."""
    ens = ch.Ensemble(descs, prec=prec, cadence=10, max_samples=nsteps // 10 + 2)
    ens.init_random()
    C0 = [ens.get_field(m) for m in range(len(descs))]
    ens.step(nsteps)
    C1 = [ens.get_field(m) for m in range(len(descs))]
    F, mC = ens.energy()
    ens.close()
    return C0, C1, F, mC


def _static(descs, prec, C0, nsteps):
    dtype = torch.float64 if prec == ch.CH_F64 else torch.float32
    field = torch.tensor(np.concatenate([c.ravel() for c in C0]), dtype=dtype, device="cuda")
    energy = torch.full((4 * len(descs),), float("nan"), dtype=torch.float64, device="cuda")
    ch.ch_step_static(descs, prec, field, nsteps, energy)
    torch.cuda.synchronize()
    out = field.double().cpu().numpy()
    S = C0[0].size
    return [out[m * S:(m + 1) * S].reshape(C0[0].shape) for m in range(len(descs))], \
        energy.cpu().numpy().reshape(-1, 4)


def _check(descs, prec, nsteps):
    C0, C1, F, mC = _reference(descs, prec, nsteps)
    got, en = _static(descs, prec, C0, nsteps)
    tol = TOL[prec]
    for m in range(len(descs)):
        err = float(np.abs(got[m] - C1[m]).max())
        print(f"static member {m} {C0[m].shape}: max|C - ctx path| = {err:.3e}", flush=True)
        assert err <= tol, (m, err)
    assert np.allclose(en[:, 0], F, rtol=1e-12, atol=0), (en[:, 0], F)
    assert np.allclose(en[:, 1], mC, rtol=0, atol=1e-12), (en[:, 1], mC)
    assert np.all(en[:, 3] == nsteps)


def test_static_matches_context_path_two_calls():
    torch.cuda.set_device(0)
    first = [ch.make_desc((64, 64), 0.01 + 0.002 * m, 1e-3, c0=0.3 * (m % 2), noise=0.05, seed=300 + m)
             for m in range(6)]
    _check(first, ch.CH_F64, 30)
    # second call on the same GPU, smaller ensemble and grid: the scratch left
    # by the first call must not leak into it
    second = [ch.make_desc((32, 48), 0.005, 5e-4, c0=-0.1, noise=0.1, seed=400 + m) for m in range(2)]
    _check(second, ch.CH_F64, 21)


def test_static_3d_fp32():
    torch.cuda.set_device(0)
    descs = [ch.make_desc((16, 16, 32), 0.01, 5e-4, c0=0.2 * m, noise=0.05, seed=500 + m) for m in range(3)]
    _check(descs, ch.CH_F32_BULK, 12)


def test_static_rejects_oversize():
    torch.cuda.set_device(0)
    field = torch.zeros(64, dtype=torch.float32, device="cuda")
    big = [ch.make_desc((1024, 1024), 0.01, 1e-3) for _ in range(32)]
    with pytest.raises(ch.ChError) as e:
        ch.ch_step_static(big, ch.CH_F32_BULK, field, 1)
    assert e.value.status == ch.CH_ENOMEM and "static scratch" in str(e.value)


@pytest.mark.parametrize("prec", [ch.CH_F64, ch.CH_F32_BULK], ids=["f64-split", "f32-wide"])
def test_static_lines_beyond_one_wavefront(prec):
    """8192-point x-lines (256 chunks over 4 wavefronts; FP64 in the split
    form, whose diagnostics come from the RHS tiles) through both paths."""
    torch.cuda.set_device(0)
    h = 2 * np.pi / 512
    descs = [ch.make_desc((8192, 8), 0.01, 5e-4, c0=0.1 * m, noise=0.1, seed=600 + m, L=(8192 * h, 8 * h))
             for m in range(2)]
    _check(descs, prec, 12)
