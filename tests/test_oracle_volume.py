"""Pins of the oracle's volume-weighted residual norm.

The volume norm integrates H^2 over the domain with the proper cell volume
dV = |h0 h1 h2| dxx0 dxx1 dxx2 (the midpoint rule on cell centres) and divides
by the domain's volume. Its pieces are pinned against closed forms that do not
involve the coordinate maps:

* the total volume of each domain: a ball of radius rmax (Spherical) or amax
  (SinhSpherical), and for SinhSymTP the prolate spheroid bounded by xx0 = 1,
  whose meridian is the ellipse with semi-axes amax (rho) and
  sqrt(amax^2 + b^2) (z), volume 4 pi a^2 c / 3;
* the mean of x^2 + y^2 + z^2 over an ellipsoid with semi-axes (a, a, c):
  (2 a^2 + c^2) / 5 (3 R^2 / 5 for a ball);
* a field that is nonzero on one cell only: its mean is its value times that
  cell's share of the volume;
* the midpoint rule converges at second order as the grid is refined.
The norm itself must equal the square root of the volume mean of H^2 with H the
oracle's own residual (pinned elsewhere against the Hamiltonian constraint).
"""
import numpy as np
import pytest

SINH_MILD = dict(amax=3.0, sinhwaa=0.4, bscale=0.5)
SSPH_MILD = dict(amax=3.0, sinhwaa=0.4)
SPH = dict(rmax=2.0)


def _axes(coords, kw):
    """Semi-axes (a, c) of the domain: a in x and y, c along z."""
    if coords == 0:
        return kw["amax"], np.hypot(kw["amax"], kw["bscale"])
    R = kw["rmax"] if coords == 1 else kw["amax"]
    return R, R


CASES = [(0, SINH_MILD), (1, SPH), (2, SSPH_MILD)]


@pytest.mark.parametrize("coords,kw", CASES)
def test_constant_field_has_unit_mean(oracle_lib, coords, kw):
    g = oracle_lib.OracleGrid(coords, 16, 12, 8, 8, **kw)
    m, vol = g.volume_mean(np.full(g.shape, 1.0))
    assert abs(m - 1.0) < 1e-14
    assert vol > 0


@pytest.mark.parametrize("coords,kw", CASES)
def test_domain_volume_and_second_moment_converge(oracle_lib, coords, kw):
    a, c = _axes(coords, kw)
    V = 4.0 * np.pi * a * a * c / 3.0
    M2 = (2.0 * a * a + c * c) / 5.0
    errs_v, errs_m = [], []
    for n in (16, 32, 64):
        g = oracle_lib.OracleGrid(coords, n, n, 8, 8, **kw)
        X, Y, Z = g.cart()
        m, vol = g.volume_mean(X * X + Y * Y + Z * Z)
        errs_v.append(abs(vol / V - 1.0))
        errs_m.append(abs(m / M2 - 1.0))
    # second-order midpoint rule: each halving of the cell width divides the
    # error by about four
    assert errs_v[-1] < 2e-3 and errs_m[-1] < 2e-3
    for e in (errs_v, errs_m):
        for k in range(2):
            assert e[k + 1] < e[k] / 3.0, e


def test_ball_volume_matches_midpoint_sums(oracle_lib):
    """Spherical: the midpoint sums of r^2 sin(theta) dr dtheta dphi have closed
    forms, sum_i r_i^2 dr = R^3/3 - R dr^2/12 and
    sum_j sin(theta_j) dtheta = 2 (dtheta/2) / sin(dtheta/2), so the oracle's
    total volume must match their product to rounding."""
    R, N0, N1, N2 = 2.0, 20, 14, 6
    g = oracle_lib.OracleGrid(1, N0, N1, N2, 8, rmax=R)
    dr, dth = R / N0, np.pi / N1
    radial = R ** 3 / 3.0 - R * dr * dr / 12.0
    polar = 2.0 * (dth / 2.0) / np.sin(dth / 2.0)
    exact = radial * polar * 2.0 * np.pi
    _, vol = g.volume_mean(np.full(g.shape, 1.0))
    assert abs(vol / exact - 1.0) < 1e-13


@pytest.mark.parametrize("coords,kw", CASES)
def test_single_cell_field_weights_by_cell_volume(oracle_lib, coords, kw):
    """A field nonzero on one interior cell (and on ghost points, which must be
    ignored) has mean f * J dV / V with J = |h0 h1 h2| at that cell's centre."""
    g = oracle_lib.OracleGrid(coords, 16, 12, 8, 8, **kw)
    ng = g.NG
    x0, x1 = g.xx(0), g.xx(1)
    f = np.zeros(g.shape)
    f[:ng, :, :] = 7.0   # ghosts in phi
    f[:, :, :ng] = 7.0   # inner ghosts in xx0
    i0, i1, i2 = ng + 5, ng + 3, ng + 2
    f[i2, i1, i0] = 2.5
    _, V = g.volume_mean(np.full(g.shape, 1.0))
    m, _ = g.volume_mean(f)
    h = g.scale_factors(x0[i0], x1[i1])
    dV = np.prod(g.dxx())
    assert abs(m - 2.5 * abs(np.prod(h)) * dV / V) < 1e-15 * 2.5


@pytest.mark.parametrize("coords,kw", CASES)
def test_residual_volume_is_root_volume_mean_of_H2(oracle_lib, coords, kw):
    g = oracle_lib.OracleGrid(coords, 16, 12, 8, 8, **kw)
    g.set_punctures([0.5, 0.5], [[0, 0, 0.4], [0, 0, -0.4]],
                    [[0.1, 0, 0], [-0.1, 0, 0]], [[0, 0, 0.1], [0, 0, 0]])
    rng = np.random.default_rng(3)
    u = g.pad_interior(0.01 * rng.standard_normal(g.N[::-1]))
    g.set_state(u, np.zeros(g.shape))
    r_pts, H = g.residual(want_H=True)
    r_vol = g.residual_volume()
    m, _ = g.volume_mean(H * H)
    assert abs(r_vol - np.sqrt(m)) <= 1e-14 * r_vol
    # the two norms weight the cells differently: they must not coincide
    assert abs(r_vol - r_pts) > 1e-3 * r_pts


def test_integration_radius_on_cell_faces_is_exact(oracle_lib):
    """Spherical with the integration radius on a cell face (r = 10 dr): the
    cells kept are exactly those of the smaller ball, so the total volume is the
    same closed-form midpoint sum taken over [0, R]."""
    rmax, N0, N1, N2 = 2.0, 20, 14, 6
    g = oracle_lib.OracleGrid(1, N0, N1, N2, 8, rmax=rmax)
    dr, dth = rmax / N0, np.pi / N1
    R = 10 * dr
    exact = (R ** 3 / 3.0 - R * dr * dr / 12.0) * 2.0 * (dth / 2.0) / np.sin(dth / 2.0) * 2.0 * np.pi
    m, vol = g.volume_mean(np.full(g.shape, 1.0), radius=R)
    assert abs(vol / exact - 1.0) < 1e-13 and abs(m - 1.0) < 1e-14
    # a radius beyond the domain keeps every cell
    _, vall = g.volume_mean(np.full(g.shape, 1.0))
    _, vbig = g.volume_mean(np.full(g.shape, 1.0), radius=10 * rmax)
    assert vbig == vall


@pytest.mark.parametrize("coords,kw", [(0, SINH_MILD), (2, SSPH_MILD)])
def test_integration_sphere_volume_and_moment_converge(oracle_lib, coords, kw):
    """A sphere of radius 1.5 inside the stretched domains (outer radius 3):
    its volume 4 pi R^3/3 and the mean of r^2 over it, 3 R^2/5, are approached
    as the grid is refined (the cells are cut at the sphere by their centres,
    so the error falls at first order or better)."""
    R = 1.5
    V, M2 = 4.0 * np.pi * R ** 3 / 3.0, 3.0 * R * R / 5.0
    ev, em = [], []
    for n in (16, 32, 64):
        g = oracle_lib.OracleGrid(coords, n, n, 16, 8, **kw)
        X, Y, Z = g.cart()
        m, vol = g.volume_mean(X * X + Y * Y + Z * Z, radius=R)
        ev.append(abs(vol / V - 1.0))
        em.append(abs(m / M2 - 1.0))
    assert ev[-1] < 0.05 and em[-1] < 0.05, (ev, em)
    assert ev[-1] < ev[0] / 2.0 and em[-1] < em[0] / 2.0, (ev, em)
