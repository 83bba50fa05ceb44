"""Pins of the oracle's finite differences and curvilinear Laplacian.

Finite differences: centred weights of order p = fd_order must be exact on
polynomials (the defining property), and equal the rationals obtained by
solving the moment (Vandermonde) system exactly with Python fractions, a
different algorithm from the oracle's Fornberg recursion.

Laplacian (flat metric in SinhSymTP / Spherical, paper "Basic equations"
section): applied to closed-form functions, its error must converge at the
stencil's order p away from the coordinate singularities (the focal
segment / origin and the axis), and at order >= p - 2 in the max norm over the
whole grid (there the coefficients grow like 1/A and 1/(A sin xx1)^2); the
exact-polynomial cases (r^2 in Spherical) must be exact to roundoff.
"""
from fractions import Fraction

import numpy as np
import pytest


def exact_weights(ng: int, deriv: int):
    """Solve sum_k w_k k^j = j! delta_{j,deriv}, j = 0..2ng, exactly."""
    offs = list(range(-ng, ng + 1))
    n = len(offs)
    A = [[Fraction(k) ** j for k in offs] for j in range(n)]
    b = [Fraction(0)] * n
    fact = 1
    for i in range(1, deriv + 1):
        fact *= i
    b[deriv] = Fraction(fact)
    # Gauss-Jordan elimination over the rationals
    M = [row[:] + [b[i]] for i, row in enumerate(A)]
    for c in range(n):
        piv = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[piv] = M[piv], M[c]
        pv = M[c][c]
        M[c] = [x / pv for x in M[c]]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c]
                M[r] = [x - f * y for x, y in zip(M[r], M[c])]
    return [M[i][n] for i in range(n)]


@pytest.mark.parametrize("order", [2, 4, 6, 8, 10])
def test_fd_weights_match_exact_rationals(oracle_lib, order):
    w1, w2 = oracle_lib.fd_weights(order)
    e1 = exact_weights(order // 2, 1)
    e2 = exact_weights(order // 2, 2)
    np.testing.assert_allclose(w1, [float(x) for x in e1], rtol=0, atol=4e-15)
    np.testing.assert_allclose(w2, [float(x) for x in e2], rtol=0, atol=4e-15)


def test_fd_weights_known_centre_values(oracle_lib):
    # Textbook values of the centre and nearest weights (order 8 and 10).
    w1, w2 = oracle_lib.fd_weights(8)
    assert abs(w2[4] - (-205 / 72)) < 1e-15 and abs(w1[5] - 0.8) < 1e-15
    w1, w2 = oracle_lib.fd_weights(10)
    assert abs(w2[5] - (-5269 / 1800)) < 1e-15 and abs(w1[6] - 5 / 6) < 1e-15


@pytest.mark.parametrize("order", [2, 4, 8, 10])
def test_fd_weights_exact_on_polynomials(oracle_lib, order):
    ng = order // 2
    w1, w2 = oracle_lib.fd_weights(order)
    k = np.arange(-ng, ng + 1, dtype=float)
    for j in range(order + 1):
        m1 = float(np.dot(w1, k ** j))
        m2 = float(np.dot(w2, k ** j))
        assert abs(m1 - (1.0 if j == 1 else 0.0)) < 1e-11, (j, m1)
        assert abs(m2 - (2.0 if j == 2 else 0.0)) < 1e-11, (j, m2)
    # the stencil is not exact one degree further (it is of order p, not more)
    j = order + 2
    assert abs(float(np.dot(w2, k ** j))) > 1e-3


def test_fornberg_nonuniform_three_point(oracle_lib):
    # Three-point weights on x = (-1, 0, 2) at z = 0 solve the 3x3 moment system.
    w = oracle_lib.fornberg(0.0, [-1.0, 0.0, 2.0], 2)
    x = np.array([-1.0, 0.0, 2.0])
    V = np.vstack([x ** 0, x, x ** 2])
    for d in range(3):
        rhs = np.zeros(3)
        rhs[d] = [1, 1, 2][d]
        np.testing.assert_allclose(V @ w[d], rhs, atol=1e-14)


SINH_MILD = dict(amax=3.0, sinhwaa=0.4, bscale=0.5)


def _r2(x, y, z):
    return x * x + y * y + z * z, 6.0 + 0.0 * x


def _gauss(x, y, z):
    r2 = (x - 0.1) ** 2 + (y + 0.2) ** 2 + (z - 0.3) ** 2
    return np.exp(-r2), (4.0 * r2 - 6.0) * np.exp(-r2)


def _inv_dist(x, y, z):
    # harmonic away from its pole, which sits off the grid points
    d = np.sqrt((x - 4.1) ** 2 + (y - 4.4) ** 2 + (z - 4.7) ** 2)
    return 1.0 / d, 0.0 * x


def _lap_errors(oracle_lib, coords, N, order, fn, kw, region):
    g = oracle_lib.OracleGrid(coords, N, N, N, order, **kw)
    X, Y, Z = g.cart()
    F, L = fn(X, Y, Z)
    e = np.abs(g.interior(g.laplacian(F)) - g.interior(L))
    if region == "all":
        return e.max()
    x0 = g.xx(0)[g.NG:g.NG + N]
    x1 = g.xx(1)[g.NG:g.NG + N]
    m0 = (x0 > 0.25 * x0.max()) & (x0 < 0.75 * x0.max())
    # away from the axis (and, for SinhCylindrical, from the z caps)
    m1 = np.abs(x1) < 0.75 if coords == 3 else np.sin(x1) > 0.5
    mask = np.broadcast_to(m1[None, :, None] & m0[None, None, :], e.shape)
    return e[mask].max()


@pytest.mark.parametrize("coords,kw", [(0, SINH_MILD), (1, dict(rmax=3.0)),
                                       (2, dict(amax=3.0, sinhwaa=0.4)),
                                       (3, dict(amax=3.0, sinhwaa=0.4))])
@pytest.mark.parametrize("order", [4, 8, 10])
@pytest.mark.parametrize("fn", [_gauss, _inv_dist])
def test_laplacian_converges_at_stencil_order(oracle_lib, coords, kw, order, fn):
    # N = 32 -> 64 is in the asymptotic range for these smooth functions
    e1 = _lap_errors(oracle_lib, coords, 32, order, fn, kw, "regular")
    e2 = _lap_errors(oracle_lib, coords, 64, order, fn, kw, "regular")
    rate = np.log2(e1 / e2)
    assert rate > order - 1.5, (e1, e2, rate)


@pytest.mark.parametrize("order", [4, 8, 10])
def test_laplacian_global_order_at_least_p_minus_2(oracle_lib, order):
    e1 = _lap_errors(oracle_lib, 0, 12, order, _gauss, SINH_MILD, "all")
    e2 = _lap_errors(oracle_lib, 0, 24, order, _gauss, SINH_MILD, "all")
    assert np.log2(e1 / e2) > order - 2 - 0.5


def test_laplacian_sinhsymtp_r2_converges(oracle_lib):
    e1 = _lap_errors(oracle_lib, 0, 24, 8, _r2, SINH_MILD, "regular")
    e2 = _lap_errors(oracle_lib, 0, 48, 8, _r2, SINH_MILD, "regular")
    assert np.log2(e1 / e2) > 7.0


@pytest.mark.parametrize("order", [2, 8, 10])
def test_laplacian_spherical_r2_is_exact(oracle_lib, order):
    # r^2 is a polynomial of degree 2 in r and independent of the angles
    e = _lap_errors(oracle_lib, 1, 16, order, _r2, dict(rmax=3.0), "all")
    assert e < 1e-10


def test_laplacian_of_cartesian_x_and_z_vanish(oracle_lib):
    # x and z are harmonic; errors must shrink at the stencil order
    for fn in (lambda x, y, z: (x, 0 * x), lambda x, y, z: (z, 0 * x)):
        e1 = _lap_errors(oracle_lib, 0, 24, 8, fn, SINH_MILD, "regular")
        e2 = _lap_errors(oracle_lib, 0, 48, 8, fn, SINH_MILD, "regular")
        assert e2 < 1e-6 and np.log2(e1 / e2) > 6.5
