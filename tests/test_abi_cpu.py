"""Host-only checks of libch.so: exported symbols, argument validation (which
runs before any device call), and the line-solve factorisation coefficients.
No GPU is needed."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1911_03386_amd import ch

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "ch.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ch_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = ch.load()
    names = header_functions()
    assert len(names) >= 18
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(ch.EXPORTED)
    assert lib.ch_version().decode().startswith("ch-mi355x")


def _desc(**kw):
    args = dict(n=(64, 64), gamma=0.01, dt=1e-3)
    args.update(kw)
    return ch.make_desc(**args)


def test_workspace_bytes_valid():
    a = ch.ch_workspace_bytes([_desc()], ch.CH_F64, 10, 11)
    b = ch.ch_workspace_bytes([_desc()], ch.CH_F32_BULK, 10, 11)
    assert a > 2 * 64 * 64 * 8 and b > 2 * 64 * 64 * 4 and a > b
    mixed = [_desc(n=(256, 256)), _desc(n=(512, 512)), _desc(n=(32, 16, 8))]
    assert ch.ch_workspace_bytes(mixed, ch.CH_F32_BULK, 10, 501) > 0


@pytest.mark.parametrize("kw,frag", [
    (dict(n=(7, 64)), "unsupported"),
    (dict(n=(64, 4100)), "unsupported"),
    (dict(n=(66, 64)), "unsupported"),
    (dict(n=(260, 64)), "unsupported"),
    (dict(gamma=0.0), "gamma"),
    (dict(dt=float("nan")), "gamma"),
    (dict(L=(2.0, -1.0)), "L > 0"),
])
def test_workspace_bytes_rejects(kw, frag):
    with pytest.raises(ch.ChError) as e:
        ch.ch_workspace_bytes([_desc(**kw)])
    assert frag in str(e.value)


@pytest.mark.parametrize("n,prec", [((8192, 8192), ch.CH_F64), ((8192, 64), ch.CH_F32_BULK),
                                    ((64, 8192), ch.CH_F64), ((2048, 1024), ch.CH_F64),
                                    ((16, 8192, 8), ch.CH_F64)])
def test_workspace_bytes_accepts_long_lines(n, prec):
    """x-lines beyond 64 chunks (2D) and columns of up to 256 chunks."""
    sites = int(np.prod(n))
    assert ch.ch_workspace_bytes([_desc(n=n)], prec, 10, 2) > 2 * sites * (8 if prec == ch.CH_F64 else 4)


@pytest.mark.parametrize("n", [(8192, 16, 8), (6144, 64), (16384, 8), (64, 16384)])
def test_workspace_bytes_rejects_lines_without_a_shape(n):
    # 3D x-lines stay within one wavefront (n <= 4096); 6144 = 64 * 4 * 24 has
    # no compiled chunk length; 16384 exceeds both line forms
    with pytest.raises(ch.ChError) as e:
        ch.ch_workspace_bytes([_desc(n=n)])
    assert "unsupported" in str(e.value)


def test_workspace_bytes_rejects_global_args():
    lib = ch.load()
    arr = ch.desc_array([_desc()])
    assert lib.ch_workspace_bytes(arr, 1, 0, 0, 10) == 0
    assert "cadence" in ch.last_error()
    assert lib.ch_workspace_bytes(arr, 1, 0, 10, 0) == 0
    assert "max_samples" in ch.last_error()
    assert lib.ch_workspace_bytes(arr, 0, 0, 10, 1) == 0
    assert lib.ch_workspace_bytes(arr, 1, 7, 10, 1) == 0
    bad = _desc()
    bad.dim = 4
    assert lib.ch_workspace_bytes(ch.desc_array([bad]), 1, 0, 10, 1) == 0
    bad = _desc()
    bad.n[2] = 2
    assert lib.ch_workspace_bytes(ch.desc_array([bad]), 1, 0, 10, 1) == 0


def test_create_validates_before_touching_the_device():
    lib = ch.load()
    arr = ch.desc_array([_desc()])
    nb = ch.ch_workspace_bytes([_desc()], 0, 10, 11)
    out = ctypes.c_void_p()
    # NULL out
    assert lib.ch_create(arr, 1, 0, 0, 10, 11, ctypes.c_void_p(4096), nb, None, None) == ch.CH_EINVAL
    # NULL workspace
    assert lib.ch_create(arr, 1, 0, 0, 10, 11, None, nb, None, ctypes.byref(out)) == ch.CH_EINVAL
    # misaligned workspace
    assert lib.ch_create(arr, 1, 0, 0, 10, 11, ctypes.c_void_p(4096 + 8), nb, None,
                         ctypes.byref(out)) == ch.CH_EINVAL
    assert "aligned" in ch.last_error()
    # too small
    assert lib.ch_create(arr, 1, 0, 0, 10, 11, ctypes.c_void_p(4096), nb - 1, None,
                         ctypes.byref(out)) == ch.CH_ENOMEM
    # bad energy convention
    assert lib.ch_create(arr, 1, 0, 5, 10, 11, ctypes.c_void_p(4096), nb, None,
                         ctypes.byref(out)) == ch.CH_EINVAL
    # unsupported size
    arr2 = ch.desc_array([_desc(n=(66, 64))])
    assert lib.ch_create(arr2, 1, 0, 0, 10, 11, ctypes.c_void_p(4096), nb, None,
                         ctypes.byref(out)) == ch.CH_EUNSUPPORTED
    assert out.value is None


def test_calls_on_unknown_contexts():
    lib = ch.load()
    bogus = ctypes.c_void_p(0x1000)
    assert lib.ch_step(None, 1) == ch.CH_EINVAL
    assert lib.ch_step(bogus, 1) == ch.CH_ESTATE
    assert lib.ch_destroy(bogus) == ch.CH_ESTATE
    assert lib.ch_init_random(bogus) == ch.CH_ESTATE
    n = ctypes.c_int64()
    assert lib.ch_get_step(bogus, ctypes.byref(n)) == ch.CH_ESTATE
    assert "destroyed" in ch.last_error()


# --------------------------------------------------------------------------
# The factorised line solve: coefficients from the library, recursion and
# chunk scan re-enacted in numpy, result compared with a dense solve.
# --------------------------------------------------------------------------
def _apply_factorised(coef, x, chunk):
    a1, a2, ik = coef[0], coef[1], coef[2]
    M = coef[3:7].reshape(2, 2)
    W = coef[7:11].reshape(2, 2)
    n = x.size
    P = n // chunk
    chunks = x.reshape(P, chunk)

    def run(v, s):  # causal recursion from state s = (u_-1, u_-2)
        out = np.empty_like(v)
        s0, s1 = s
        for k in range(v.size):
            u = v[k] + a1 * s0 + a2 * s1
            s1, s0 = s0, u
            out[k] = u
        return out, np.array([s0, s1])

    def solve_causal(ch_):
        E = [run(c, (0.0, 0.0))[1] for c in ch_]
        Z = np.zeros(2)
        for e in E:
            Z = M @ Z + e
        S = W @ Z
        outs = []
        for q in range(P):
            o, _ = run(ch_[q], S)
            outs.append(o)
            S = M @ S + E[q]
        return np.array(outs)

    u = solve_causal(chunks)
    # anti-causal = causal on the reversed sequence
    v = solve_causal(u.reshape(-1)[::-1].reshape(P, chunk))
    return v.reshape(-1)[::-1] * ik


@pytest.mark.parametrize("rho,n,chunk", [(1.72, 128, 8), (441.0, 64, 16), (1764.0, 64, 4),
                                         (13.8, 32, 32), (0.05, 16, 4), (1e5, 16, 8),
                                         (2.0e4, 8, 8)])
def test_factorised_solve_matches_dense(rho, n, chunk):
    coef = ch.ch_solver_coefficients(rho, n, chunk, ch.CH_F64)
    # poles inside the unit circle
    assert coef[1] < 0 and -coef[1] < 1
    A = np.eye(n)
    for i in range(n):
        for o, c in zip([-2, -1, 0, 1, 2], [1, -4, 6, -4, 1]):
            A[i, (i + o) % n] += rho * c
    rng = np.random.default_rng(int(rho) + n)
    x = rng.standard_normal(n)
    y = _apply_factorised(coef, x, chunk)
    ref = np.linalg.solve(A, x)
    assert np.abs(y - ref).max() < 1e-11 * np.abs(ref).max() * max(1.0, rho) ** 0.25
    # constants are preserved (the scheme conserves the mean)
    ones = _apply_factorised(coef, np.ones(n), chunk)
    assert np.abs(ones - 1).max() < 1e-12 * max(1.0, rho) ** 0.5


def test_factorised_solve_fp32_coefficients():
    rho, n, chunk = 441.0, 512, 16
    coef = ch.ch_solver_coefficients(rho, n, chunk, ch.CH_F32_BULK)
    assert np.float32(coef[0]) == coef[0] and np.float32(coef[1]) == coef[1]
    # DC gain is exactly one for the rounded coefficients (up to FP64 rounding)
    a1, a2, ik = coef[:3]
    assert abs(ik / (1 - a1 - a2) ** 2 - 1) < 1e-15


# ---- droplet-population ensembles (include/dp.h) -----------------------------

DP_HEADER = os.path.join(os.path.dirname(HEADER), "dp.h")


def test_library_exports_every_droplet_symbol():
    from paper_1911_03386_amd import dp

    text = re.sub(r"/\*.*?\*/", "", open(DP_HEADER).read(), flags=re.S)
    names = sorted(set(re.findall(r"\b(dp_[a-z_0-9]+)\s*\(", text)))
    assert len(names) >= 12
    lib = dp.lib()
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(dp.EXPORTED)


@pytest.mark.parametrize("n,kw,frag", [
    ([0], {}, "1 <= n"),
    ([8193], {}, "1 <= n"),
    ([16], dict(dt_sample=0.0), "dt_sample > 0"),
    ([16], dict(rtol=-1.0), "rtol > 0"),
    ([16], dict(t_end=float("inf")), "t_end >= 0"),
    ([16], dict(max_attempts=0), "max_attempts"),
])
def test_droplet_workspace_rejects(n, kw, frag):
    from paper_1911_03386_amd import dp

    args = dict(t_end=1.0)
    args.update(kw)
    with pytest.raises(dp.DpError) as e:
        dp.workspace_bytes(n, dp.make_params(**args))
    assert frag in str(e.value)


def test_droplet_workspace_grows_with_samples_and_droplets():
    from paper_1911_03386_amd import dp

    a = dp.workspace_bytes([128, 8192], dp.make_params(40.0, 0.1))
    b = dp.workspace_bytes([128, 8192], dp.make_params(80.0, 0.1))
    c = dp.workspace_bytes([128, 8192, 8192], dp.make_params(40.0, 0.1))
    assert 0 < a < b and a < c
    assert a >= 8 * (128 + 8192) + 8 * 6 * 2 * 401


def test_droplet_create_rejects_bad_workspace_before_any_device_call():
    import ctypes

    from paper_1911_03386_amd import dp

    L = dp.lib()
    prm = dp.make_params(1.0)
    n, p = dp._i32([64, 100])
    nb = dp.workspace_bytes([64, 100], prm)
    ctx = ctypes.c_void_p()
    st = L.dp_create(p, 2, ctypes.byref(prm), None, nb, None, ctypes.byref(ctx))
    assert st == dp.CH_EINVAL and "256-byte aligned" in dp.last_error()
    st = L.dp_create(p, 2, ctypes.byref(prm), ctypes.c_void_p(4096 + 8), nb, None, ctypes.byref(ctx))
    assert st == dp.CH_EINVAL and "256-byte aligned" in dp.last_error()
    st = L.dp_create(p, 2, ctypes.byref(prm), ctypes.c_void_p(4096), nb - 1, None, ctypes.byref(ctx))
    assert st == dp.CH_EINVAL and "need" in dp.last_error()
    assert ctx.value is None
    # calls on a context that does not exist are refused without touching it
    bogus = ctypes.c_void_p(0x1000)
    assert L.dp_advance(bogus, 1) == dp.CH_ESTATE
    assert L.dp_destroy(None) == dp.CH_EINVAL


class _FakeTensor:
    """Stands in for a device tensor: only its address is passed, and every
    case below is refused before the library touches the device."""

    def __init__(self, ptr):
        self._ptr = ptr

    def data_ptr(self):
        return self._ptr


class _FakeStream:
    cuda_stream = 0


@pytest.mark.parametrize("descs,ptr,nsteps,status,frag", [
    ([], 256, 1, ch.CH_EINVAL, "outside"),
    ([_desc()] * 65, 256, 1, ch.CH_EINVAL, "outside"),
    ([_desc(), _desc(n=(64, 32))], 256, 1, ch.CH_EINVAL, "grid of member 0"),
    ([_desc()], 0, 1, ch.CH_EINVAL, "NULL"),
    ([_desc()], 8, 1, ch.CH_EINVAL, "aligned"),
    ([_desc()], 256, -1, ch.CH_EINVAL, "nsteps"),
    ([_desc(n=(7, 64))], 256, 1, ch.CH_EUNSUPPORTED, "unsupported"),
    ([_desc(n=(1024, 1024))] * 32, 256, 1, ch.CH_ENOMEM, "static scratch"),
])
def test_step_static_validation(descs, ptr, nsteps, status, frag):
    with pytest.raises(ch.ChError) as e:
        ch.ch_step_static(descs, ch.CH_F32_BULK, _FakeTensor(ptr), nsteps, stream=_FakeStream())
    assert e.value.status == status and frag in str(e.value), str(e.value)
