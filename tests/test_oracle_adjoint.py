"""Pins of the oracle's velocity gradient (the discrete adjoint of the step).

The C oracle back-propagates in the z = c G ybar form; the NumPy twin holds
an independent ybar recursion and the tangent-linear model.  The dot-product
test ties the adjoint to the tangent-linear model to rounding; central finite
differences of the forward map tie both to the true derivative."""
import numpy as np
import pytest

import fd_inputs as fi
from oracle import np_twin


def _small(ndim):
    if ndim == 2:
        return fi.surface2d(22, 26, 60, seed=3).scaled(sponge_width=5, sponge_alpha=0.06)
    return fi.layered3d(nx=14, ny=12, nz=12, nt=40).scaled(sponge_width=3, sponge_alpha=0.1)


@pytest.mark.parametrize("ndim", [2, 3])
def test_adjoint_dot_product(orc, ndim):
    p = _small(ndim)
    v = fi.random_velocity(p.shape, 21)
    tw = np_twin.Twin(p, v)
    rng = np.random.default_rng(2)
    dc = rng.standard_normal(p.shape) * tw.c * 1e-2
    r = rng.standard_normal((p.nt, p.receivers.count))
    Jdc = tw.tangent(p.wavelet(), p.nt, dc)
    g = orc.grid_of(p)
    shp = (p.nz, p.ny, p.nx)
    _, gc = orc.adjoint(g, v.reshape(shp), p.wavelet(), p.nt, p.src, p.rec_index(), r)
    lhs = float(np.vdot(Jdc, r))
    rhs = float(np.vdot(dc.reshape(shp), gc))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


@pytest.mark.parametrize("ndim", [2, 3])
def test_adjoint_matches_twin_recursion(orc, ndim):
    p = _small(ndim)
    v = fi.random_velocity(p.shape, 22)
    tw = np_twin.Twin(p, v)
    r = np.random.default_rng(5).standard_normal((p.nt, p.receivers.count))
    gc_twin = tw.adjoint_c(p.wavelet(), p.nt, r)
    shp = (p.nz, p.ny, p.nx)
    gv, gc = orc.adjoint(orc.grid_of(p), v.reshape(shp), p.wavelet(), p.nt, p.src,
                         p.rec_index(), r)
    assert orc.rel_l2(gc.reshape(gc_twin.shape), gc_twin) <= 1e-12
    # dJ/dv = dJ/dc * dc/dv, c = (v dt/h)^2
    cc = tw.c
    assert orc.rel_l2(gv.reshape(gc_twin.shape), gc_twin * 2 * cc / v.astype(np.float64)) <= 1e-13


def _misfit(orc, g, v, p, dobs):
    out = orc.forward(g, v, p.wavelet(), p.nt, p.src, p.rec_index())
    res = out["traces"] - dobs
    return 0.5 * float(np.sum(res * res)), res


def test_gradient_central_differences_directional(orc):
    p = fi.surface2d(22, 26, 60, seed=3).scaled(sponge_width=5, sponge_alpha=0.06)
    shp = (p.nz, 1, p.nx)
    g = orc.grid_of(p)
    vtrue = fi.random_velocity(shp, 31, 2000, 3000)
    v0 = fi.random_velocity(shp, 32, 2000, 3000)
    dobs = orc.forward(g, vtrue, p.wavelet(), p.nt, p.src, p.rec_index())["traces"]
    _, res = _misfit(orc, g, v0, p, dobs)
    gv, _ = orc.adjoint(g, v0, p.wavelet(), p.nt, p.src, p.rec_index(), res)
    dv = fi.perturbation(shp, 33)
    # The forward consumes FP32 velocities; take the perturbation on the
    # FP64 side through c by running the twin (FP64 velocity) instead.
    tw0 = np_twin.Twin(p, v0)
    base = v0.astype(np.float64).reshape(p.shape)
    d = dv.reshape(p.shape)
    for h in (1e-1, 1e-2):
        def J(vv):
            tw0.c = (vv * p.dt / p.dh) ** 2
            tr, _, _, _ = tw0.forward(p.wavelet(), p.nt)
            rr = tr - dobs
            return 0.5 * float(np.sum(rr * rr))
        fd = (J(base + h * d) - J(base - h * d)) / (2 * h)
        an = float(np.vdot(gv.reshape(p.shape), d))
        assert abs(fd - an) <= 1e-6 * abs(an), (h, fd, an)


def test_gradient_central_differences_per_cell(orc):
    p = fi.surface2d(16, 18, 50, seed=4).scaled(sponge_width=4, sponge_alpha=0.06)
    shp = (p.nz, 1, p.nx)
    g = orc.grid_of(p)
    vtrue = fi.random_velocity(shp, 41, 2000, 3000)
    v0 = fi.random_velocity(shp, 42, 2000, 3000)
    dobs = orc.forward(g, vtrue, p.wavelet(), p.nt, p.src, p.rec_index())["traces"]
    _, res = _misfit(orc, g, v0, p, dobs)
    gv, _ = orc.adjoint(g, v0, p.wavelet(), p.nt, p.src, p.rec_index(), res)
    tw = np_twin.Twin(p, v0)
    base = v0.astype(np.float64).reshape(p.shape)
    h = 0.05
    for cell in [(3, 5), (8, 9), (12, 2), (2, 9)]:
        def J(vv):
            tw.c = (vv * p.dt / p.dh) ** 2
            tr, _, _, _ = tw.forward(p.wavelet(), p.nt)
            rr = tr - dobs
            return 0.5 * float(np.sum(rr * rr))
        vp = base.copy(); vp[cell] += h
        vm = base.copy(); vm[cell] -= h
        fd = (J(vp) - J(vm)) / (2 * h)
        an = gv.reshape(p.shape)[cell]
        assert abs(fd - an) <= 1e-6 * abs(an) + 1e-30, (cell, fd, an)
