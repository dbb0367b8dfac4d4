"""Pins of the oracle's imaging condition (reverse-time migration image).

The image is the zero-lag correlation sum_k z^k w^{k-1} of the source
wavefield and the z-form receiver wavefield; it is the derivative of
J = <r, traces> with respect to a field m of point scatterers, the spatial
operator L becoming L + diag(m).  The NumPy twin holds a forward map with
scatterers and its tangent-linear model, written separately from the C
oracle: the dot-product test ties the image to the tangent-linear model to
rounding, and central differences of the twin's forward map in m tie both to
the true derivative.  A dropped c or G factor, a one-step shift of the
correlation or a transposed operand fails these."""
import numpy as np
import pytest

import fd_inputs as fi
from oracle import np_twin


def _small(ndim):
    if ndim == 2:
        return fi.surface2d(22, 26, 60, seed=3).scaled(sponge_width=5, sponge_alpha=0.06)
    return fi.layered3d(nx=14, ny=12, nz=12, nt=40).scaled(sponge_width=3, sponge_alpha=0.1)


@pytest.mark.parametrize("ndim", [2, 3])
def test_image_dot_product_with_scatterer_tangent(orc, ndim):
    p = _small(ndim)
    v = fi.random_velocity(p.shape, 71)
    tw = np_twin.Twin(p, v)
    rng = np.random.default_rng(7)
    dm = rng.standard_normal(p.shape) * 1e-2
    r = rng.standard_normal((p.nt, p.receivers.count))
    dtr = tw.tangent_m(p.wavelet(), p.nt, dm)
    shp = (p.nz, p.ny, p.nx)
    img = orc.image(orc.grid_of(p), v.reshape(shp), p.wavelet(), p.nt, p.src, p.rec_index(), r)
    lhs = float(np.vdot(dtr, r))
    rhs = float(np.vdot(dm.reshape(shp), img))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_image_central_differences_per_cell(orc):
    p = fi.surface2d(16, 18, 50, seed=4).scaled(sponge_width=4, sponge_alpha=0.06)
    v = fi.random_velocity(p.shape, 72)
    tw = np_twin.Twin(p, v)
    r = np.random.default_rng(8).standard_normal((p.nt, p.receivers.count))
    img = orc.image(orc.grid_of(p), v.reshape(p.nz, 1, p.nx), p.wavelet(), p.nt, p.src,
                    p.rec_index(), r).reshape(p.shape)
    h = 1e-3
    # cells the wavefield reaches within the 50 steps (far cells hold values
    # near the FP64 rounding of J, where a difference quotient is noise)
    for cell in [(3, 5), (8, 9), (5, 12), (6, 15)]:
        assert abs(img[cell]) > 1e-6 * np.abs(img).max()
        m = np.zeros(p.shape)
        m[cell] = h
        jp = float(np.vdot(tw.forward_m(p.wavelet(), p.nt, m), r))
        m[cell] = -h
        jm = float(np.vdot(tw.forward_m(p.wavelet(), p.nt, m), r))
        fd = (jp - jm) / (2 * h)
        assert abs(fd - img[cell]) <= 1e-6 * abs(img[cell]) + 1e-30, (cell, fd, img[cell])


def test_image_is_linear_in_the_data(orc):
    p = _small(2)
    v = fi.random_velocity(p.shape, 73)
    shp = (p.nz, p.ny, p.nx)
    rng = np.random.default_rng(9)
    r1 = rng.standard_normal((p.nt, p.receivers.count))
    r2 = rng.standard_normal((p.nt, p.receivers.count))
    g = orc.grid_of(p)
    i1 = orc.image(g, v.reshape(shp), p.wavelet(), p.nt, p.src, p.rec_index(), r1)
    i2 = orc.image(g, v.reshape(shp), p.wavelet(), p.nt, p.src, p.rec_index(), r2)
    i12 = orc.image(g, v.reshape(shp), p.wavelet(), p.nt, p.src, p.rec_index(), 2 * r1 - 3 * r2)
    assert orc.rel_l2(i12, 2 * i1 - 3 * i2) <= 1e-13
