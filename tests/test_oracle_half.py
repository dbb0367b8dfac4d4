"""Pins of the oracle's reduced-precision emulation (FP32 arithmetic with
FP32 or 16-bit field storage).

The rounding of FP32 to binary16 and to bfloat16 is pinned bit-exactly
against two library routines (numpy's float16 cast and torch's bfloat16 cast,
both round-to-nearest-even); the FP32 arithmetic of the emulated time loop is
pinned against the NumPy twin's independent emulation.  The 16-bit
fixed-point form of the model term c is pinned by its defining properties
(scale bracket, nearest code with ties to even, cap, monotonicity), by the
twin's separate implementation, and by models whose c values are codes
already, for which it must change nothing.  The FP32-storage form is pinned
bit for bit to the FP64 scheme on inputs whose arithmetic FP32 carries out
exactly, and to rounding level on ordinary ones."""
import numpy as np
import pytest
import torch

import fd_inputs as fi
from oracle import np_twin


def _probe_values():
    rng = np.random.default_rng(0)
    parts = [
        rng.standard_normal(20000).astype(np.float32) * np.float32(10.0) ** rng.integers(-9, 6, 20000).astype(np.float32),
        np.array([0.0, -0.0, 1.0, -1.0, 65504.0, 65519.99, 65520.0, 1e6, -1e6, np.inf, -np.inf,
                  2.0 ** -14, 2.0 ** -24, 2.0 ** -25, 2.0 ** -25 * 1.0000001, 2.0 ** -26, 1e-30,
                  3.0 * 2.0 ** -26, 2.0 ** -15 + 2.0 ** -25], dtype=np.float32),
    ]
    # exact ties for binary16 normals (bit 12 set, lower bits clear) and bf16
    u = rng.integers(0x38800000, 0x477F0000, 5000, dtype=np.uint32)
    parts.append(((u & ~np.uint32(0x1FFF)) | np.uint32(0x1000)).view(np.float32))
    parts.append(((u & ~np.uint32(0xFFFF)) | np.uint32(0x8000)).view(np.float32))
    # subnormal-range binary16 values
    parts.append(rng.uniform(-2.0 ** -14, 2.0 ** -14, 5000).astype(np.float32))
    return np.concatenate(parts).astype(np.float32)


def test_f16_rounding_matches_numpy(orc):
    x = _probe_values()
    got = orc.encode(1, x)
    with np.errstate(over="ignore"):   # the probe values include overflow to inf
        ref = x.astype(np.float16).view(np.uint16)
    np.testing.assert_array_equal(got, ref)
    back = orc.decode(1, ref)
    np.testing.assert_array_equal(back, ref.view(np.float16).astype(np.float32))


def test_bf16_rounding_matches_torch(orc):
    x = _probe_values()
    x = x[np.isfinite(x)]
    got = orc.encode(2, x)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    np.testing.assert_array_equal(got, ref)
    back = orc.decode(2, ref)
    np.testing.assert_array_equal(
        back, torch.from_numpy(ref.view(np.int16)).view(torch.bfloat16).float().numpy())


@pytest.mark.parametrize("storage", [1, 2])
@pytest.mark.parametrize("ndim", [2, 3])
def test_half_emulation_matches_twin(orc, storage, ndim):
    if ndim == 2:
        p = fi.surface2d(26, 30, 70, seed=8).scaled(sponge_width=4, sponge_alpha=0.06)
    else:
        p = fi.layered3d(nx=14, ny=13, nz=12, nt=40)
    v = fi.random_velocity(p.shape, 17)
    shp = (p.nz, p.ny, p.nx)
    out = orc.forward_half(orc.grid_of(p), storage, v.reshape(shp), p.wavelet(), p.nt, p.src,
                           p.rec_index())
    tr, cur = np_twin.Twin(p, v).forward_half(p.wavelet(), p.nt, storage)
    # Same FP32 operation order and rounding on both sides: bit-identical.
    np.testing.assert_array_equal(out["traces"], tr)
    np.testing.assert_array_equal(out["cur"].reshape(cur.shape), cur)


@pytest.mark.parametrize("storage,bound", [(1, 2e-3), (2, 3e-2)])
def test_half_error_against_fp64_is_bounded(orc, storage, bound):
    p = fi.surface2d(48, 52, 150, seed=9)
    v = fi.random_velocity(p.shape, 18, 2000, 3500)
    shp = (p.nz, 1, p.nx)
    g = orc.grid_of(p)
    ref = orc.forward(g, v.reshape(shp), p.wavelet(), p.nt, p.src, p.rec_index())
    out = orc.forward_half(g, storage, v.reshape(shp), p.wavelet(), p.nt, p.src, p.rec_index())
    e_tr = orc.rel_l2(out["traces"], ref["traces"])
    e_f = orc.rel_l2(out["cur"], ref["cur"])
    assert e_tr <= bound and e_f <= bound, (e_tr, e_f)
    # 16-bit storage must cost more than FP32 rounding alone
    assert e_f > 1e-6


def test_c_fixed16_codes_are_nearest_with_ties_to_even(orc):
    rng = np.random.default_rng(21)
    c = rng.uniform(0.01, 0.2, 50000).astype(np.float32)
    c[0] = np.float32(0.2)                       # the largest value
    q, e, dec = orc.c_fixed16(c)
    M = float(c.max())
    assert 2.0 ** (e - 1) <= M < 2.0 ** e        # the scale brackets the largest c
    t = c.astype(np.float64) * 2.0 ** (16 - e)
    qf = q.astype(np.float64)
    assert np.all(np.abs(qf - t) <= 0.5)          # nearest code
    assert np.all(np.abs(dec.astype(np.float64) - c) <= 2.0 ** (e - 17))
    np.testing.assert_array_equal(dec.astype(np.float64), qf * 2.0 ** (e - 16))
    order = np.argsort(c, kind="stable")
    assert np.all(np.diff(qf[order]) >= 0)        # monotone
    # exact midpoints between codes round to the even code
    k = rng.integers(1000, 60000, 2000).astype(np.float64)
    mid = np.concatenate([[M], (k + 0.5) * 2.0 ** (e - 16)]).astype(np.float32)
    assert np.all(mid.astype(np.float64)[1:] == (k + 0.5) * 2.0 ** (e - 16))
    qm, em, _ = orc.c_fixed16(mid)
    assert em == e
    assert np.all(qm[1:] % 2 == 0)
    assert np.all(np.abs(qm[1:].astype(np.float64) - (k + 0.5)) == 0.5)


def test_c_fixed16_top_of_bracket_and_powers_of_two(orc):
    # a largest c within half a code of a power of two would round to 2^16
    # in its own bracket: the scale moves up one binade, and the error bound
    # 2^(e-17) holds for that value too
    top = np.nextafter(np.float32(0.25), np.float32(0.0))
    vals = np.array([top, 0.125, 0.0625, 0.0], dtype=np.float32)
    q, e, dec = orc.c_fixed16(vals)
    assert e == -1 and q[0] == 32768
    assert q[1] == 16384 and q[2] == 8192 and q[3] == 0
    assert np.all(np.abs(dec.astype(np.float64) - vals) <= 2.0 ** (e - 17))
    # just below that band the bracket stays: the largest code is 65535
    t = np.float32((65535.25) * 2.0 ** -18)
    q, e, dec = orc.c_fixed16(np.array([t, 0.1], dtype=np.float32))
    assert e == -2 and q[0] == 65535
    assert abs(float(dec[0]) - float(t)) <= 2.0 ** (e - 17)
    # a largest c that is a power of two sits at the bottom of its bracket
    q, e, _ = orc.c_fixed16(np.array([0.125, 0.03125], dtype=np.float32))
    assert e == -2 and q[0] == 32768 and q[1] == 8192


@pytest.mark.parametrize("storage", [1, 2])
@pytest.mark.parametrize("ndim", [2, 3])
def test_c_fixed16_emulation_matches_twin(orc, storage, ndim):
    if ndim == 2:
        p = fi.surface2d(26, 30, 70, seed=8).scaled(sponge_width=4, sponge_alpha=0.06)
    else:
        p = fi.layered3d(nx=14, ny=13, nz=12, nt=40)
    v = fi.random_velocity(p.shape, 17)
    shp = (p.nz, p.ny, p.nx)
    out = orc.forward_half(orc.grid_of(p), storage, v.reshape(shp), p.wavelet(), p.nt, p.src,
                           p.rec_index(), c_fixed16=True)
    tr, cur = np_twin.Twin(p, v).forward_half(p.wavelet(), p.nt, storage, c_fixed16=True)
    np.testing.assert_array_equal(out["traces"], tr)
    np.testing.assert_array_equal(out["cur"].reshape(cur.shape), cur)
    plain = orc.forward_half(orc.grid_of(p), storage, v.reshape(shp), p.wavelet(), p.nt, p.src,
                             p.rec_index())
    assert not np.array_equal(plain["cur"], out["cur"])   # the option takes effect


@pytest.mark.parametrize("storage", [1, 2])
def test_c_fixed16_changes_nothing_when_c_is_a_code(orc, storage):
    # dt/dh = 1e-4: v = 2500 gives c = 1/16, v = 1250 gives c = 1/64, both
    # codes of the fixed-point grid (e = -3)
    p = fi.surface2d(30, 34, 60, seed=8).scaled(dt=1e-3, dh=10.0)
    v = np.full(p.shape, 2500.0, dtype=np.float32)
    v[p.nz // 2:] = 1250.0
    shp = (p.nz, 1, p.nx)
    g = orc.grid_of(p)
    a = orc.forward_half(g, storage, v.reshape(shp), p.wavelet(), p.nt, p.src, p.rec_index())
    b = orc.forward_half(g, storage, v.reshape(shp), p.wavelet(), p.nt, p.src, p.rec_index(),
                         c_fixed16=True)
    np.testing.assert_array_equal(a["traces"], b["traces"])
    np.testing.assert_array_equal(a["cur"], b["cur"])


@pytest.mark.parametrize("storage,bound", [(1, 2e-3), (2, 3e-2)])
def test_c_fixed16_error_against_fp64_is_bounded(orc, storage, bound):
    p = fi.surface2d(48, 52, 150, seed=9)
    v = fi.random_velocity(p.shape, 18, 2000, 3500)
    shp = (p.nz, 1, p.nx)
    g = orc.grid_of(p)
    ref = orc.forward(g, v.reshape(shp), p.wavelet(), p.nt, p.src, p.rec_index())
    out = orc.forward_half(g, storage, v.reshape(shp), p.wavelet(), p.nt, p.src, p.rec_index(),
                           c_fixed16=True)
    assert orc.rel_l2(out["traces"], ref["traces"]) <= bound
    assert orc.rel_l2(out["cur"], ref["cur"]) <= bound


# --------------------------------------------------------------------------
# FP32 storage (storage 0): the scheme with nothing but FP32 rounding, the
# floor against which FP32 GPU results are judged at sizes the FP64 oracle
# only samples.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("ndim", [2, 3])
def test_f32_emulation_matches_twin(orc, ndim):
    if ndim == 2:
        p = fi.surface2d(26, 30, 70, seed=8).scaled(sponge_width=4, sponge_alpha=0.06)
    else:
        p = fi.layered3d(nx=14, ny=13, nz=12, nt=40)
    v = fi.random_velocity(p.shape, 17)
    shp = (p.nz, p.ny, p.nx)
    out = orc.forward_half(orc.grid_of(p), 0, v.reshape(shp), p.wavelet(), p.nt, p.src, p.rec_index())
    tr, cur = np_twin.Twin(p, v).forward_half(p.wavelet(), p.nt, 0)
    np.testing.assert_array_equal(out["traces"], tr)
    np.testing.assert_array_equal(out["cur"].reshape(cur.shape), cur)


@pytest.mark.parametrize("ndim", [2, 3])
def test_f32_emulation_is_exact_where_the_arithmetic_is(orc, ndim):
    """With radius 1 (weights -2, 1), c = 1/16 (v dt / dh = 1/4 exactly), no
    damping and a unit impulse at step 0 (amplitude dt^2/dh^D = 2^-20), every
    value of the first steps is a dyadic rational short enough for FP32, so
    FP32 arithmetic rounds nothing and must give the FP64 scheme bit for bit.
    A dropped or mis-signed term, a wrong weight or a shifted index in the
    FP32 loop would show here exactly."""
    n = 17
    shape = (n, n) if ndim == 2 else (n, n, n)
    p = fi.Problem(name="dyadic", ndim=ndim, nz=n, ny=1 if ndim == 2 else n, nx=n, dh=1.0,
                   dt=2.0 ** -10, nt=6, src=(8, 0 if ndim == 2 else 7, 9),
                   receivers=fi.Receivers(8, 0, 0, 1, 1, n), f0=10.0, radius=1,
                   sponge_width=0, velocity_kind="constant", v_const=256.0)
    g = orc.grid_of(p)
    v = np.full((p.nz, p.ny, p.nx), 256.0, dtype=np.float32)
    wav = np.zeros(p.nt, dtype=np.float32)
    wav[0] = 1.0
    ref = orc.forward(g, v, wav, p.nt, p.src, p.rec_index())
    out = orc.forward_half(g, 0, v, wav, p.nt, p.src, p.rec_index())
    # precondition: the FP64 values are FP32 numbers (no rounding anywhere)
    assert np.array_equal(ref["cur"].astype(np.float32).astype(np.float64), ref["cur"])
    assert np.count_nonzero(ref["cur"]) > 80   # 85 (2D) and 377 (3D) cells reached
    np.testing.assert_array_equal(out["cur"].astype(np.float64), ref["cur"])
    np.testing.assert_array_equal(out["traces"].astype(np.float64), ref["traces"])


@pytest.mark.parametrize("ndim", [2, 3])
def test_f32_emulation_against_fp64_is_at_rounding_level(orc, ndim):
    """Against the FP64 scheme on a sponge-damped random model the FP32
    emulation stays at rounding level (measured: 2D 5.5e-7 traces / 1.6e-6
    field after 150 steps; 3D 4.2e-7 / 2.7e-7 after 80 steps): a bound of 1e-5, far
    below what any wrong term would give and above the growth of rounding
    error with the step count."""
    if ndim == 2:
        p = fi.surface2d(48, 52, 150, seed=9)
        v = fi.random_velocity(p.shape, 18, 2000, 3500)
    else:
        p = fi.layered3d(nx=24, ny=22, nz=20, nt=80)
        v = fi.random_velocity(p.shape, 19, 1500, 4500)
    shp = (p.nz, p.ny, p.nx)
    g = orc.grid_of(p)
    ref = orc.forward(g, v.reshape(shp), p.wavelet(), p.nt, p.src, p.rec_index())
    out = orc.forward_half(g, 0, v.reshape(shp), p.wavelet(), p.nt, p.src, p.rec_index())
    e_tr = orc.rel_l2(out["traces"], ref["traces"])
    e_f = orc.rel_l2(out["cur"], ref["cur"])
    print(f"FP32 emulation vs FP64 ({ndim}D): traces {e_tr:.2e} field {e_f:.2e}")
    assert e_tr <= 1e-5 and e_f <= 1e-5, (e_tr, e_f)
    assert e_f > 0.0   # FP32 rounding does show


def test_f32_emulation_rejects_16bit_c(orc):
    p = fi.surface2d(20, 20, 5, seed=1)
    v = fi.random_velocity(p.shape, 2)
    with pytest.raises(ValueError):
        orc.forward_half(orc.grid_of(p), 0, v.reshape(p.nz, 1, p.nx), p.wavelet(), p.nt, p.src,
                         p.rec_index(), c_fixed16=True)
