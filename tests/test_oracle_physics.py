"""Pins of the oracle's time stepping against what the equation fixes.

Eq. 1 (Section 7) with a constant velocity and a point source has closed
Green's functions in 2D and in 3D (the same equation with a third axis); the
leapfrog scheme of the step order in Listing 3 conserves a discrete energy
with symmetric L and no damping; the scheme is reciprocal after scaling by c.
Each is checked in 2D and in 3D, and each would fail for a dropped term, a
wrong sign, a wrong source scaling (dt^2/dh^D) or a shifted time index."""
import math

import numpy as np
import pytest
from scipy import integrate

import fd_inputs as fi
from oracle import np_twin


def _ricker(t, f0):
    a = (math.pi * f0 * (t - 1.5 / f0)) ** 2
    return (1 - 2 * a) * math.exp(-a)


def green2d_pressure(r, t, v, f0):
    """P(r, t) = 1/(2 pi v^2) * int_0^{acosh(vt/r)} s(t - (r/v) cosh th) dth:
    the time convolution of the 2D Green's function H(vt-r)/(2 pi v sqrt(v^2 t^2 - r^2))
    with the source, after substituting v tau = r cosh th."""
    if v * t <= r:
        return 0.0
    up = math.acosh(v * t / r)
    val, _ = integrate.quad(lambda th: _ricker(t - (r / v) * math.cosh(th), f0), 0.0, up,
                            limit=200)
    return val / (2 * math.pi * v * v)


def _green_errors(orc, prob):
    g = orc.grid_of(prob)
    out = orc.forward(g, prob.velocity(), prob.wavelet(), prob.nt, prob.src, prob.rec_index())
    errs = []
    # The source is added before the derivatives, so off-source trace row n
    # approximates P at t = (n + 2) dt.
    ts = (np.arange(prob.nt) + 2) * prob.dt
    for off in (10, 20, 30):
        ref = np.array([green2d_pressure(off * prob.dh, t, prob.v_const, prob.f0) for t in ts])
        errs.append(orc.rel_l2(out["traces"][:, prob.src[2] + off], ref))
    return np.array(errs)


def test_green_function_2d_and_dt_convergence(orc):
    p = fi.green2d()
    e1 = _green_errors(orc, p)
    assert np.all(e1 <= 5e-3), e1
    e2 = _green_errors(orc, p.scaled(dt=p.dt / 2, nt=p.nt * 2))
    ratio = e1 / e2
    assert np.all(ratio >= 3.5), ratio


def test_green_function_wrong_time_index_fails(orc):
    # The same comparison at t = (n+1) dt must be much worse: the pin is
    # sensitive to the source timing.
    p = fi.green2d()
    g = orc.grid_of(p)
    out = orc.forward(g, p.velocity(), p.wavelet(), p.nt, p.src, p.rec_index())
    ts = (np.arange(p.nt) + 1) * p.dt
    ref = np.array([green2d_pressure(200.0, t, 2000.0, 15.0) for t in ts])
    assert orc.rel_l2(out["traces"][:, 148], ref) > 2e-2


def _energy(orc, g, prev, cur, c):
    Lprev = orc.laplacian(g, prev)
    return float(np.sum((cur - prev) ** 2 / c) - np.sum(cur * Lprev))


@pytest.mark.parametrize("bc", [0, 1])
def test_discrete_energy_conserved(orc, bc):
    shape = (96, 1, 80)
    p = fi.Problem(name="energy", ndim=2, nz=96, ny=1, nx=80, dh=10.0, dt=1e-3, nt=0,
                   src=(40, 0, 30), receivers=fi.Receivers(0, 0, 0, 1, 1, 1), f0=25.0,
                   bc=bc, sponge_width=0)
    g = orc.grid_of(p)
    v = fi.random_velocity(shape, 5)
    c, _ = orc.setup(g, v)
    w = fi.ricker(25.0, 1e-3, 200)
    w[120:] = 0.0     # the source stops; energy is conserved from then on
    out = orc.forward(g, v, w, 200, p.src, [0])
    prev, cur = out["prev"], out["cur"]
    E0 = _energy(orc, g, prev, cur, c)
    assert E0 > 0
    zero = np.zeros(10, dtype=np.float32)
    Es = []
    for _ in range(26):
        out = orc.forward(g, v, zero, 100, None, [0], init_prev=prev, init_cur=cur)
        prev, cur = out["prev"], out["cur"]
        Es.append(_energy(orc, g, prev, cur, c))
    Es = np.array(Es)
    assert np.all(Es > 0)
    assert np.abs(Es - E0).max() <= 1e-12 * E0


def test_energy_grows_above_cfl_limit(orc):
    # 2D limit C = sqrt(4 / (2 * 6.50159)) = 0.5546; at C = 0.57 the scheme blows up.
    n = 40
    shape = (n, 1, n)
    dt = 0.57 * 10.0 / 3000.0
    p = fi.Problem(name="cfl", ndim=2, nz=n, ny=1, nx=n, dh=10.0, dt=dt, nt=0,
                   src=(20, 0, 20), receivers=fi.Receivers(0, 0, 0, 1, 1, 1), f0=20.0)
    g = orc.grid_of(p)
    v = np.full(shape, 3000.0, dtype=np.float32)
    rng = np.random.default_rng(0)
    cur = rng.standard_normal(shape) * 1e-6
    out = orc.forward(g, v, np.zeros(1, np.float32), 400, None, [0], init_prev=cur, init_cur=cur)
    assert np.abs(out["cur"]).max() > 1e3
    dt_ok = 0.54 * 10.0 / 3000.0
    g2 = orc.grid_of(p.scaled(dt=dt_ok))
    out = orc.forward(g2, v, np.zeros(1, np.float32), 400, None, [0], init_prev=cur, init_cur=cur)
    assert np.abs(out["cur"]).max() < 1e-4


def test_reciprocity(orc):
    shape = (40, 1, 48)
    v = fi.random_velocity(shape, 9)
    p = fi.Problem(name="recip", ndim=2, nz=40, ny=1, nx=48, dh=10.0, dt=1e-3, nt=150,
                   src=(10, 0, 12), receivers=fi.Receivers(0, 0, 0, 1, 1, 1), f0=20.0)
    g = orc.grid_of(p)
    c, _ = orc.setup(g, v)
    s, r = (10, 0, 12), (27, 0, 35)
    lin = lambda q: (q[0] * 1 + q[1]) * 48 + q[2]
    w = p.wavelet()
    tr_sr = orc.forward(g, v, w, 150, s, [lin(r)])["traces"][:, 0]
    tr_rs = orc.forward(g, v, w, 150, r, [lin(s)])["traces"][:, 0]
    cs, cr = c.ravel()[lin(s)], c.ravel()[lin(r)]
    assert orc.rel_l2(cs * tr_sr, cr * tr_rs) <= 1e-12
    assert orc.rel_l2(tr_sr, tr_rs) > 1e-3   # the c scaling matters here


def test_sponge_absorbs(orc):
    n = 64
    p = fi.Problem(name="absorb", ndim=2, nz=n, ny=1, nx=n, dh=10.0, dt=1e-3, nt=0,
                   src=(32, 0, 32), receivers=fi.Receivers(0, 0, 0, 1, 1, 1), f0=25.0,
                   sponge_width=16, sponge_faces=fi.FACES_ALL)
    g = orc.grid_of(p)
    v = np.full((n, 1, n), 2500.0, dtype=np.float32)
    w = fi.ricker(25.0, 1e-3, 100)
    out = orc.forward(g, v, w, 100, p.src, [0])
    peak = float(np.sum(out["cur"] ** 2))
    out2 = orc.forward(g, v, np.zeros(1, np.float32), 700, None, [0],
                       init_prev=out["prev"], init_cur=out["cur"])
    assert float(np.sum(out2["cur"] ** 2)) < 1e-2 * peak
    # without the band the energy stays trapped by the zero edges
    g0 = orc.grid_of(p.scaled(sponge_width=0))
    out = orc.forward(g0, v, w, 100, p.src, [0])
    out2 = orc.forward(g0, v, np.zeros(1, np.float32), 700, None, [0],
                       init_prev=out["prev"], init_cur=out["cur"])
    assert float(np.sum(out2["cur"] ** 2)) > 1e-1 * float(np.sum(out["cur"] ** 2))


@pytest.mark.parametrize("ndim", [2, 3])
def test_forward_matches_numpy_twin(orc, ndim):
    if ndim == 2:
        p = fi.surface2d(30, 34, 60, seed=1).scaled(sponge_width=5, sponge_alpha=0.05)
    else:
        p = fi.layered3d(nx=18, ny=16, nz=14, nt=40)
    v = fi.random_velocity(p.shape, 4)
    g = orc.grid_of(p)
    vv = v.reshape(p.nz, p.ny, p.nx)
    out = orc.forward(g, vv, p.wavelet(), p.nt, p.src, p.rec_index())
    tw = np_twin.Twin(p, v)
    tr, cur, prev, _ = tw.forward(p.wavelet(), p.nt)
    assert orc.rel_l2(out["traces"], tr) <= 1e-13
    assert orc.rel_l2(out["cur"].reshape(cur.shape), cur) <= 1e-13
    assert orc.rel_l2(out["prev"].reshape(prev.shape), prev) <= 1e-13


# --------------------------------------------------------------------------
# 3D: the same pins on the three-axis scheme
# --------------------------------------------------------------------------

def green3d_pressure(r, t, v, f0):
    """P(r, t) = s(t - r/v) / (4 pi v^2 r): the source convolved with the 3D
    free-space Green's function delta(t - r/v) / (4 pi v^2 r) of
    P_tt - v^2 lap P = S(t) delta(x)."""
    return _ricker(t - r / v, f0) / (4.0 * math.pi * v * v * r)


# receiver offsets from the source, in cells (z, y, x): along each axis, both
# signs, and one body diagonal
_OFFS3 = [(0, 0, 10), (0, -15, 0), (20, 0, 0), (-12, 0, 0), (8, 8, 8)]


def _green3d_errors(orc, dt, nt, shift=2):
    """Oracle traces on an 81^3 homogeneous grid (v = 2000 m/s, dh = 10 m,
    15 Hz Ricker at the centre cell) against the closed form at the receiver
    offsets above.  The nearest edge is 40 cells from the source, so no
    reflection reaches a receiver (offset <= 20 cells) before the last
    sample at 0.28 s."""
    n, v, h, f0 = 81, 2000.0, 10.0, 15.0
    c = n // 2
    p = fi.Problem(name="green3d", ndim=3, nz=n, ny=n, nx=n, dh=h, dt=dt, nt=nt,
                   src=(c, c, c), receivers=fi.Receivers(0, 0, 0, 1, 1, 1), f0=f0,
                   sponge_width=0, velocity_kind="constant", v_const=v)
    lin = [((c + o[0]) * n + c + o[1]) * n + c + o[2] for o in _OFFS3]
    out = orc.forward(orc.grid_of(p), p.velocity(), p.wavelet(), nt, p.src, lin)
    ts = (np.arange(nt) + shift) * dt
    errs = []
    for k, o in enumerate(_OFFS3):
        r = h * math.sqrt(o[0] ** 2 + o[1] ** 2 + o[2] ** 2)
        ref = np.array([green3d_pressure(r, t, v, f0) for t in ts])
        errs.append(orc.rel_l2(out["traces"][:, k], ref))
    return np.array(errs)


def test_green_function_3d_and_dt_convergence(orc):
    # dt = 0.5 ms, 560 steps (0.28 s); then dt halved.  Measured errors at
    # 100-200 m: 0.8-1.8e-3, dropping 3.8-4.5x on halving dt (the time
    # discretisation dominates; the diagonal keeps a little anisotropic
    # spatial error).  A source scaled dt^2/dh^2 (the 2D factor) would be off
    # by a factor dh = 10, and one at t = (n+1) dt by ~5%.
    e1 = _green3d_errors(orc, 5e-4, 560)
    assert np.all(e1 <= 5e-3), e1
    e2 = _green3d_errors(orc, 2.5e-4, 1120)
    ratio = e1 / e2
    assert np.all(ratio >= 3.5), ratio


def test_green_function_3d_wrong_time_index_fails(orc):
    e = _green3d_errors(orc, 5e-4, 560, shift=1)
    assert np.all(e > 2e-2), e


def _problem3d(shape, dt, bc=0, src=(5, 6, 7)):
    nz, ny, nx = shape
    return fi.Problem(name="p3", ndim=3, nz=nz, ny=ny, nx=nx, dh=10.0, dt=dt, nt=0, src=src,
                      receivers=fi.Receivers(0, 0, 0, 1, 1, 1), f0=25.0, bc=bc,
                      sponge_width=0)


@pytest.mark.parametrize("bc", [0, 1])
def test_discrete_energy_conserved_3d(orc, bc):
    shape = (22, 18, 20)
    p = _problem3d(shape, 8e-4, bc=bc, src=(9, 8, 11))
    g = orc.grid_of(p)
    v = fi.random_velocity(shape, 15)
    c, _ = orc.setup(g, v)
    w = fi.ricker(25.0, 8e-4, 120)
    w[80:] = 0.0     # the source stops; energy is conserved from then on
    out = orc.forward(g, v, w, 120, p.src, [0])
    prev, cur = out["prev"], out["cur"]
    E0 = _energy(orc, g, prev, cur, c)
    assert E0 > 0
    zero = np.zeros(10, dtype=np.float32)
    Es = []
    for _ in range(12):
        out = orc.forward(g, v, zero, 60, None, [0], init_prev=prev, init_cur=cur)
        prev, cur = out["prev"], out["cur"]
        Es.append(_energy(orc, g, prev, cur, c))
    Es = np.array(Es)
    assert np.all(Es > 0)
    assert np.abs(Es - E0).max() <= 1e-12 * E0


def test_energy_grows_above_cfl_limit_3d(orc):
    # 3D limit C = sqrt(4 / (3 * 6.50159)) = 0.45286: at C = 0.47 the scheme
    # blows up, at C = 0.44 it stays bounded.
    n = 20
    shape = (n, n, n)
    v = np.full(shape, 3000.0, dtype=np.float32)
    rng = np.random.default_rng(1)
    cur = rng.standard_normal(shape) * 1e-6
    for C, grows in ((0.47, True), (0.44, False)):
        p = _problem3d(shape, C * 10.0 / 3000.0)
        out = orc.forward(orc.grid_of(p), v, np.zeros(1, np.float32), 400, None, [0],
                          init_prev=cur, init_cur=cur)
        big = np.abs(out["cur"]).max()
        assert (big > 1e3) if grows else (big < 1e-4), (C, big)


def test_reciprocity_3d(orc):
    shape = (18, 20, 22)
    v = fi.random_velocity(shape, 19)
    p = _problem3d(shape, 8e-4)
    p = p.scaled(f0=20.0)
    g = orc.grid_of(p)
    c, _ = orc.setup(g, v)
    s, r = (4, 5, 6), (13, 12, 15)
    lin = lambda q: (q[0] * shape[1] + q[1]) * shape[2] + q[2]
    w = fi.ricker(20.0, 8e-4, 150)
    tr_sr = orc.forward(g, v, w, 150, s, [lin(r)])["traces"][:, 0]
    tr_rs = orc.forward(g, v, w, 150, r, [lin(s)])["traces"][:, 0]
    cs, cr = c.ravel()[lin(s)], c.ravel()[lin(r)]
    assert orc.rel_l2(cs * tr_sr, cr * tr_rs) <= 1e-12
    assert orc.rel_l2(tr_sr, tr_rs) > 1e-3   # the c scaling matters here
