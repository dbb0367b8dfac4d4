"""Pins of the oracle's spatial operator against what mathematics fixes.

The paper (Section 7, Listing 3) names the second-derivative routines but not
their order or weights; the 8th-order (R = 4) central weights are pinned here
by exact-rational moment conditions, by their known truncation constant, by
exactness on polynomials and by symmetry."""
from fractions import Fraction
import math

import numpy as np
import pytest

from oracle import np_twin


@pytest.mark.parametrize("R", [1, 2, 3, 4])
def test_closed_form_weights_solve_moment_system(orc, R):
    exact = np_twin.weights_exact(R)
    got = orc.coefficients(R)
    for k in range(R + 1):
        assert abs(got[k] - float(exact[k])) <= 1e-15 * max(1.0, abs(float(exact[k])))


def test_eighth_order_weights_textbook_values(orc):
    # Central 8th-order second-derivative weights (Fornberg, Math. Comp. 1988).
    ref = [Fraction(-205, 72), Fraction(8, 5), Fraction(-1, 5), Fraction(8, 315), Fraction(-1, 560)]
    assert np_twin.weights_exact(4) == ref
    got = orc.coefficients(4)
    np.testing.assert_allclose(got, [float(x) for x in ref], rtol=0, atol=1e-15)


def test_low_order_weights(orc):
    np.testing.assert_allclose(orc.coefficients(1), [-2.0, 1.0], atol=0)
    np.testing.assert_allclose(orc.coefficients(2), [-2.5, 4.0 / 3.0, -1.0 / 12.0], atol=1e-15)


def test_truncation_constant_degree_ten():
    # sum_k a_|k| k^10 = 10! * (leading error coefficient -1/3150) = -1152
    a = np_twin.weights_exact(4)
    m10 = a[0] * 0 + sum(2 * a[k] * k ** 10 for k in range(1, 5))
    assert m10 == -1152
    assert Fraction(math.factorial(10)) * Fraction(-1, 3150) == -1152
    for m in range(0, 5):
        mm = (a[0] if m == 0 else 0) + sum(2 * a[k] * k ** (2 * m) for k in range(1, 5))
        assert mm == (2 if m == 1 else 0)


def test_symbol_monotone_and_range(orc):
    a = orc.coefficients(4)
    th = np.linspace(0, np.pi, 2001)
    sym = a[0] + 2 * sum(a[k] * np.cos(k * th) for k in range(1, 5))
    assert abs(sym[0]) < 1e-14
    assert np.all(np.diff(sym) < 1e-15)
    exact_min = np_twin.weights_exact(4)[0] + sum(
        2 * w * (-1) ** k for k, w in enumerate(np_twin.weights_exact(4)) if k > 0)
    assert abs(sym[-1] - float(exact_min)) < 1e-13
    assert abs(sym[-1] + 6.5015873) < 1e-7


def _grid(orc, ndim, nz, ny, nx, bc=0):
    return orc.OrGrid(ndim=ndim, radius=4, bc=bc, sponge_width=0, nz=nz, ny=ny, nx=nx,
                      dh=1.0, dt=1.0, sponge_alpha=0.0, sponge_faces=0)


@pytest.mark.parametrize("p,q", [(0, 0), (2, 0), (0, 2), (9, 0), (0, 9), (5, 4), (9, 9), (7, 3)])
def test_polynomial_exactness_2d(orc, p, q):
    nz, nx = 21, 23
    z = np.arange(nz, dtype=np.float64) - 10
    x = np.arange(nx, dtype=np.float64) - 11
    Z, X = np.meshgrid(z, x, indexing="ij")
    u = X ** p * Z ** q
    exact = (p * (p - 1) * X ** max(p - 2, 0) * Z ** q if p >= 2 else 0 * u) + \
            (q * (q - 1) * X ** p * Z ** max(q - 2, 0) if q >= 2 else 0 * u)
    Lu = orc.laplacian(_grid(orc, 2, nz, 1, nx), u.reshape(nz, 1, nx)).reshape(nz, nx)
    inner = (slice(4, nz - 4), slice(4, nx - 4))
    scale = np.abs(u[inner]).max() * 16 + 1.0
    assert np.abs(Lu[inner] - exact[inner]).max() <= 1e-13 * scale


@pytest.mark.parametrize("p,q,r", [(9, 0, 0), (0, 9, 0), (0, 0, 9), (3, 4, 2), (2, 2, 2), (9, 9, 9)])
def test_polynomial_exactness_3d(orc, p, q, r):
    n = 13
    c = np.arange(n, dtype=np.float64) - 6
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")

    def d2(e, A):
        return e * (e - 1) * A ** max(e - 2, 0) if e >= 2 else 0 * A
    u = X ** p * Y ** q * Z ** r
    exact = d2(p, X) * Y ** q * Z ** r + X ** p * d2(q, Y) * Z ** r + X ** p * Y ** q * d2(r, Z)
    Lu = orc.laplacian(_grid(orc, 3, n, n, n), u)
    inner = (slice(4, n - 4),) * 3
    scale = np.abs(u).max() * 20 + 1.0
    assert np.abs(Lu[inner] - exact[inner]).max() <= 1e-13 * scale


def test_degree_ten_gives_truncation_constant(orc):
    nz, nx = 9, 41
    x = np.arange(nx, dtype=np.float64) - 20
    u = np.tile(x ** 10, (nz, 1))
    Lu = orc.laplacian(_grid(orc, 2, nz, 1, nx), u.reshape(nz, 1, nx)).reshape(nz, nx)
    # exact second derivative of x^10 vanishes at x = 0; the stencil gives -1152
    assert abs(Lu[4, 20] - (-1152.0)) < 1e-6


@pytest.mark.parametrize("ndim,bc", [(2, 0), (2, 1), (3, 0), (3, 1)])
def test_laplacian_symmetric(orc, ndim, bc):
    rng = np.random.default_rng(7)
    shape = (17, 1, 19) if ndim == 2 else (11, 12, 13)
    g = _grid(orc, ndim, *shape, bc=bc)
    u = rng.standard_normal(shape)
    w = rng.standard_normal(shape)
    lhs = np.vdot(orc.laplacian(g, u), w)
    rhs = np.vdot(u, orc.laplacian(g, w))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1)


@pytest.mark.parametrize("ndim,bc", [(2, 0), (2, 1), (3, 0), (3, 1)])
def test_laplacian_matches_numpy_twin(orc, ndim, bc):
    rng = np.random.default_rng(11)
    shape = (15, 1, 18) if ndim == 2 else (9, 10, 11)
    u = rng.standard_normal(shape)
    got = orc.laplacian(_grid(orc, ndim, *shape, bc=bc), u)
    uu = u.reshape(shape[0], shape[2]) if ndim == 2 else u
    ref = np_twin.laplacian(uu, 4, periodic=bool(bc)).reshape(shape)
    assert np.abs(got - ref).max() <= 1e-13


def test_laplacian_zero_edges_is_zero_padding(orc):
    # Brute force: zero edges equal the periodic operator on a zero-padded grid.
    rng = np.random.default_rng(3)
    u = rng.standard_normal((10, 1, 12))
    got = orc.laplacian(_grid(orc, 2, 10, 1, 12), u)
    pad = np.zeros((10 + 8, 1, 12 + 8))
    pad[4:14, :, 4:16] = u
    ref = orc.laplacian(_grid(orc, 2, 18, 1, 20, bc=1), pad)[4:14, :, 4:16]
    assert np.abs(got - ref).max() <= 1e-13


def test_sponge_profile_shape(orc):
    # Band of width W on the low face only: g = exp(-(alpha d)^2), d = W - i.
    W, alpha, n = 8, 0.3 / 8, 30
    g = orc.sponge_profile(n, W, alpha, True, False)
    assert g[0] == pytest.approx(math.exp(-0.09), rel=1e-15)
    assert np.all(g[W:] == 1.0)
    assert np.all(np.diff(g[: W + 1]) > 0)
    gh = orc.sponge_profile(n, W, alpha, False, True)
    np.testing.assert_array_equal(gh, g[::-1])
