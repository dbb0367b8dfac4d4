"""Pins of the damping band ("sponge") in the oracle.

How the damping enters the update, new = G (2 P + c L P) - G^2 Pold, is pinned
by an exact identity: for a spatially uniform G = g, Q^n = P^n / g^n obeys the
undamped scheme, so the damped run from (Pold, P) equals g^n times the
undamped run from (g Pold, P), field by field and trace by trace (FP64, from
random start states, no source).  A damping factor on the wrong term or with
the wrong power breaks it at the size of 1 - g.  The profile itself,
g = exp(-(alpha d)^2) with d the distance into the band, is a reading of what
the paper leaves open; its properties are checked: 1 off the band, strictly
decreasing into it, only on enabled faces, and the 3D field G the product of
the axis profiles."""
import numpy as np
import pytest

import fd_inputs as fi
import oracle


def _problem(ndim):
    if ndim == 2:
        return fi.surface2d(30, 34, 50, seed=2)
    return fi.layered3d(nx=14, ny=13, nz=12, nt=40)


@pytest.mark.parametrize("ndim", [2, 3])
def test_uniform_damping_is_a_rescaled_undamped_run(orc, ndim):
    p = _problem(ndim)
    shp = (p.nz, p.ny, p.nx)
    v = fi.random_velocity(p.shape, 5, 2000, 3000).reshape(shp)
    g = orc.grid_of(p)
    rng = np.random.default_rng(7)
    prev0, cur0 = rng.standard_normal(shp), rng.standard_normal(shp)
    gval, nt, rec = 0.97, p.nt, p.rec_index()
    damped = orc.forward_G(g, v, np.full(shp, gval), nt, prev0, cur0, rec)
    plain = orc.forward_G(g, v, np.ones(shp), nt, gval * prev0, cur0, rec)
    scale = max(np.abs(plain["cur"]).max(), np.abs(plain["traces"]).max())
    tol = 1e-11 * scale
    np.testing.assert_allclose(damped["cur"], gval ** nt * plain["cur"], rtol=0, atol=tol)
    np.testing.assert_allclose(damped["prev"], gval ** (nt - 1) * plain["prev"], rtol=0, atol=tol)
    steps = gval ** np.arange(1, nt + 1)
    np.testing.assert_allclose(damped["traces"], steps[:, None] * plain["traces"], rtol=0, atol=tol)
    # the damping is not a no-op at this size
    assert np.abs(damped["cur"] - plain["cur"]).max() > 0.1 * np.abs(plain["cur"]).max()


def test_given_damping_field_reproduces_the_band(orc):
    p = _problem(2).scaled(sponge_width=6, sponge_alpha=0.05)
    shp = (p.nz, p.ny, p.nx)
    v = fi.random_velocity(p.shape, 6, 2000, 3000).reshape(shp)
    g = orc.grid_of(p)
    rng = np.random.default_rng(8)
    prev0, cur0 = rng.standard_normal(shp), rng.standard_normal(shp)
    _, G = orc.setup(g, v)
    a = orc.forward_G(g, v, G, p.nt, prev0, cur0, p.rec_index())
    b = orc.forward(g, v, np.zeros(p.nt, np.float32), p.nt, None, p.rec_index(), init_prev=prev0,
                    init_cur=cur0)
    np.testing.assert_array_equal(a["cur"], b["cur"])
    np.testing.assert_array_equal(a["traces"], b["traces"])


@pytest.mark.parametrize("n,width", [(50, 8), (20, 9), (9, 4)])
def test_profile_properties(orc, n, width):
    alpha = 0.3 / width
    both = orc.sponge_profile(n, width, alpha, True, True)
    lo = orc.sponge_profile(n, width, alpha, True, False)
    hi = orc.sponge_profile(n, width, alpha, False, True)
    off = orc.sponge_profile(n, width, alpha, False, False)
    assert np.all(off == 1.0)
    assert np.all(orc.sponge_profile(n, 0, alpha, True, True) == 1.0)
    for prof in (both, lo, hi):
        assert np.all((prof > 0) & (prof <= 1))
    # lower face: 1 from index `width` on, strictly increasing up to it
    assert np.all(lo[width:] == 1.0) and np.all(np.diff(lo[:width + 1]) > 0)
    # upper face: the mirror image
    np.testing.assert_array_equal(hi, lo[::-1])
    # both faces: the smaller of the two at every cell
    np.testing.assert_array_equal(both, np.minimum(lo, hi))


def test_3d_damping_field_is_the_product_of_axis_profiles(orc):
    p = fi.layered3d(nx=20, ny=18, nz=16, nt=4).scaled(sponge_width=5, sponge_alpha=0.07)
    shp = (p.nz, p.ny, p.nx)
    g = orc.grid_of(p)
    _, G = orc.setup(g, fi.random_velocity(p.shape, 9, 2000, 3000).reshape(shp))
    f = p.sponge_faces
    gz = orc.sponge_profile(p.nz, 5, 0.07, bool(f & 1), bool(f & 2))
    gy = orc.sponge_profile(p.ny, 5, 0.07, bool(f & 4), bool(f & 8))
    gx = orc.sponge_profile(p.nx, 5, 0.07, bool(f & 16), bool(f & 32))
    np.testing.assert_allclose(G, gz[:, None, None] * gy[None, :, None] * gx[None, None, :], rtol=1e-15)
    assert G.min() < 0.9                       # the band damps
    assert G[p.nz - 1, p.ny // 2, p.nx // 2] < 1 and G[0, p.ny // 2, p.nx // 2] == 1   # no top face
