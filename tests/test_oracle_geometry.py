"""Pins of the oracle's coordinates, scale factors, Laplacian coefficients,
ghost-zone images and wave speed.

* Scale factors h_i must equal |d x_cart / d xx_i| of the oracle's own
  Cartesian map (a separately coded function), and the coordinate lines must be
  orthogonal (the Laplacian is written for a diagonal metric).
* The first-derivative coefficients b_i = (1/J) d_i (J / h_i^2), J = h0 h1 h2,
  must match a numerical derivative built from the scale factors alone.
* Every ghost point's image (parity reflections and phi periodicity) must sit at
  the same Cartesian position, and be an interior or outer point.
* The variable wave speed keeps the local Courant number c dt / ds_min at
  kappa * CFL everywhere (end of the "Basic equations" section).
"""
import numpy as np
import pytest

SINH = dict(amax=1.0e6, sinhwaa=0.07, bscale=1.0)
SINH_MILD = dict(amax=3.0, sinhwaa=0.4, bscale=0.5)
SSPH = dict(amax=1.0e6, sinhwaa=0.07)          # SinhSpherical
SSPH_MILD = dict(amax=3.0, sinhwaa=0.4)
SCYL = dict(amax=1.0e6, sinhwaa=0.07)          # SinhCylindrical
SCYL_MILD = dict(amax=3.0, sinhwaa=0.4)


def _grid(oracle_lib, coords, kw, N=(16, 12, 8), order=8):
    return oracle_lib.OracleGrid(coords, *N, order, **kw)


def _jac(g, x0, x1, x2, eps):
    J = np.zeros((3, 3))
    base = [x0, x1, x2]
    for d in range(3):
        p = list(base)
        m = list(base)
        p[d] += eps[d]
        m[d] -= eps[d]
        J[:, d] = (g.to_cart(*p) - g.to_cart(*m)) / (2 * eps[d])
    return J


COORDS = [(0, SINH_MILD), (0, SINH), (1, dict(rmax=100.0)), (2, SSPH_MILD), (2, SSPH),
          (3, SCYL_MILD), (3, SCYL), (4, dict(rmax=2.0))]


@pytest.mark.parametrize("coords,kw", COORDS)
def test_scale_factors_match_jacobian_and_orthogonality(oracle_lib, coords, kw):
    g = _grid(oracle_lib, coords, kw)
    rng = np.random.default_rng(1)
    x0max = kw["rmax"] if coords == 1 else 1.0
    for _ in range(25):
        x0 = rng.uniform(0.05, 0.95) * x0max
        x1 = rng.uniform(-0.95, 0.95) if coords == 3 else rng.uniform(0.1, np.pi - 0.1)
        x2 = rng.uniform(-np.pi, np.pi)
        eps = [1e-6 * x0max, 1e-6, 1e-6]
        J = _jac(g, x0, x1, x2, eps)
        h = g.scale_factors(x0, x1)
        cols = np.linalg.norm(J, axis=0)
        np.testing.assert_allclose(np.abs(h), cols, rtol=2e-7)
        G = J.T @ J
        off = np.abs(G - np.diag(np.diag(G))).max()
        assert off < 2e-6 * np.abs(np.diag(G)).max()


@pytest.mark.parametrize("coords,kw", COORDS)
def test_laplacian_coefficients_from_scale_factors(oracle_lib, coords, kw):
    g = _grid(oracle_lib, coords, kw, N=(16, 12, 4))
    met = g.metric()
    x0s = g.xx(0)
    x1s = g.xx(1)
    ng = g.NG
    for i1 in range(ng, ng + 12, 3):
        for i0 in range(ng, ng + 16, 3):
            x0, x1 = x0s[i0], x1s[i1]
            h = g.scale_factors(x0, x1)
            a = 1.0 / h ** 2

            def J_over_h2(d, y0, y1):
                hh = g.scale_factors(y0, y1)
                return np.prod(hh) / hh[d] ** 2

            e0 = 1e-5 * max(abs(x0), 1e-3)
            e1 = 1e-5
            b0 = (J_over_h2(0, x0 + e0, x1) - J_over_h2(0, x0 - e0, x1)) / (2 * e0) / np.prod(h)
            b1 = (J_over_h2(1, x0, x1 + e1) - J_over_h2(1, x0, x1 - e1)) / (2 * e1) / np.prod(h)
            np.testing.assert_allclose(met["a0"][i1, i0], a[0], rtol=1e-12)
            np.testing.assert_allclose(met["a1"][i1, i0], a[1], rtol=1e-12)
            np.testing.assert_allclose(met["a2"][i1, i0], a[2], rtol=1e-12)
            # with SinhCylindrical at amax 1e6, w 0.07, J/h0^2 = Z' A/A' is flat
            # to 1/cosh^2(xx0/w) where xx0 >> w, so its numerical derivative
            # keeps few digits there; the mild-parameter case pins b0
            if not (coords == 3 and kw["amax"] > 1e3):
                np.testing.assert_allclose(met["b0"][i1, i0], b0, rtol=1e-7)
            np.testing.assert_allclose(met["b1"][i1, i0], b1, rtol=1e-7)


def test_sinhsymtp_foci_and_compactification(oracle_lib):
    g = _grid(oracle_lib, 0, dict(amax=1.0e6, sinhwaa=0.07, bscale=5.0))
    # xx0 = 0 collapses onto the focal segment |z| <= b on the axis
    assert np.allclose(g.to_cart(0.0, 0.0, 0.3), [0, 0, 5.0], atol=1e-12)
    assert np.allclose(g.to_cart(0.0, np.pi, 0.3), [0, 0, -5.0], atol=1e-12)
    # xx0 = 1 is the outer boundary at radius ~ amax
    p = g.to_cart(1.0, 1.0, 0.2)
    assert abs(np.linalg.norm(p) / 1.0e6 - 1.0) < 1e-9


@pytest.mark.parametrize("coords,kw,N", [(0, SINH, (8, 6, 4)), (1, dict(rmax=10.0), (8, 6, 4)),
                                         (0, SINH_MILD, (5, 5, 6)), (1, dict(rmax=3.0), (5, 5, 2)),
                                         (2, SSPH, (8, 6, 4)), (2, SSPH_MILD, (5, 5, 6)),
                                         (3, SCYL, (8, 6, 4)), (3, SCYL_MILD, (5, 5, 6))])
def test_ghost_images_share_cartesian_position(oracle_lib, coords, kw, N):
    g = oracle_lib.OracleGrid(coords, *N, 8, **kw)
    img = g.bc_images()
    X, Y, Z = [a.reshape(-1) for a in g.cart()]
    ghosts = np.nonzero(img >= 0)[0]
    assert len(ghosts) > 0
    im = img[ghosts]
    scale = max(np.abs(X).max(), np.abs(Z).max())
    d = np.sqrt((X[ghosts] - X[im]) ** 2 + (Y[ghosts] - Y[im]) ** 2 + (Z[ghosts] - Z[im]) ** 2)
    assert d.max() < 1e-12 * scale
    # images are interior (-1) or outer (-2) points, never other ghosts
    assert np.all(img[im] < 0)
    # every point is classified
    assert np.all(img != -3)
    nint = int(np.sum(img == -1))
    nout = int(np.sum(img == -2))
    ng = g.NG
    assert nint == N[0] * N[1] * N[2]
    if coords == 3:
        # the xx0 face, and both z faces over the interior and outer xx0 range
        assert nout == ng * N[1] * N[2] + 2 * ng * (N[0] + ng) * N[2]
    else:
        assert nout == ng * N[1] * N[2]


def test_sinhspherical_radius_and_origin(oracle_lib):
    g = _grid(oracle_lib, 2, SSPH)
    # r = A(xx0): xx0 = 1 is the outer sphere r = amax, xx0 = 0 the origin
    for x1, x2 in ((0.3, 1.0), (2.0, -2.5)):
        np.testing.assert_allclose(np.linalg.norm(g.to_cart(1.0, x1, x2)), 1.0e6, rtol=1e-12)
        assert np.linalg.norm(g.to_cart(0.0, x1, x2)) == 0.0
    # the same sinh stretching as SinhSymTP's A (b = 0 there gives the same map)
    h = _grid(oracle_lib, 0, dict(amax=1.0e6, sinhwaa=0.07, bscale=1e-300))
    for x0 in (0.1, 0.5, 0.9):
        np.testing.assert_allclose(np.linalg.norm(g.to_cart(x0, 0.7, 0.1)),
                                   np.linalg.norm(h.to_cart(x0, 0.7, 0.1)), rtol=1e-12)


def test_wave_speed_gives_uniform_courant_number(oracle_lib):
    g = _grid(oracle_lib, 0, SINH, N=(32, 16, 4))
    met = g.metric()
    dsmin = met["dsmin"]
    ng = g.NG
    inter = dsmin[ng:ng + 16, ng:ng + 32]
    assert abs(inter.min() - g.ds_g()) == 0.0
    dt = g.suggest_dt(0.5)
    kappa = 1.0
    c = kappa * inter / g.ds_g()
    np.testing.assert_allclose(c * dt / inter, 0.5 * kappa, rtol=1e-14)
    # the compactified grid spans many decades of cell size
    assert inter.max() / inter.min() > 1e5


def test_sinhcylindrical_map(oracle_lib):
    """rho = A(xx0) and z = A(xx1) with the sinh stretching of SinhSymTP's A:
    xx0 = 1 is the cylinder rho = amax, xx1 = +-1 its caps z = +-amax, xx0 = 0
    the z axis, and z is odd in xx1."""
    g = _grid(oracle_lib, 3, SCYL)
    for x1, x2 in ((0.3, 1.0), (-0.7, -2.5)):
        p = g.to_cart(1.0, x1, x2)
        np.testing.assert_allclose(np.hypot(p[0], p[1]), 1.0e6, rtol=1e-12)
        q = g.to_cart(0.0, x1, x2)
        assert q[0] == 0.0 and q[1] == 0.0
    for x0, x2 in ((0.2, 0.4), (0.9, -1.0)):
        np.testing.assert_allclose(g.to_cart(x0, 1.0, x2)[2], 1.0e6, rtol=1e-12)
        np.testing.assert_allclose(g.to_cart(x0, -1.0, x2)[2], -1.0e6, rtol=1e-12)
    h = _grid(oracle_lib, 2, SSPH)   # SinhSpherical's r is the same A
    for x in (0.1, 0.5, 0.9):
        np.testing.assert_allclose(g.to_cart(0.3, x, 0.2)[2],
                                   np.linalg.norm(h.to_cart(x, 0.7, 0.1)), rtol=1e-12)
        np.testing.assert_allclose(g.to_cart(0.3, -x, 0.2)[2], -g.to_cart(0.3, x, 0.2)[2],
                                   rtol=1e-15)
