"""Pins of the oracle's Cartesian-like family (the cube [-rmax, rmax]^3,
x0, x1, x2 = x, y, z, outer boundary on all six faces).

* Classification: the NG-deep slab beyond each face holds the outer points
  (exactly one coordinate beyond the cube); edge and corner points (two or
  three beyond) are neither read by the star stencil nor by a face point's
  normal difference, and stay unused; there are no parity images.
* Brill-Lindquist punctures (no momenta, no spins) give a zero source, so
  u = v = 0 stays exactly zero.
* The equal-mass configuration with opposite momenta along y is symmetric
  under x -> -x and under the half turn (y, z) -> (-y, -z); on the
  cell-centred cube these are index reversals, and the relaxed u must have
  them to rounding.
* Laplacian: on the uniform cube the order-p centred second difference is
  exact on polynomials of degree <= p + 1 along each axis (x^k + y^k + z^k) and
  not beyond; on a Gaussian its error falls at about order p under
  refinement.
(The radiation condition on the faces is pinned in ``test_oracle_pins.py``,
the steady state against Newton's method in ``test_oracle_relax.py``.)
"""
import numpy as np
import pytest

CART = dict(rmax=6.0)


@pytest.mark.parametrize("order", [2, 4, 8, 10])
def test_laplacian_exact_on_polynomials(oracle_lib, order):
    g = oracle_lib.OracleGrid(oracle_lib.CARTESIAN, 12, 10, 8, order, rmax=1.5)
    X, Y, Z = g.cart()
    for k in range(order + 3):
        F = X ** k + Y ** k + Z ** k
        L = k * (k - 1) * (X ** max(k - 2, 0) + Y ** max(k - 2, 0) + Z ** max(k - 2, 0))
        err = np.abs(g.interior(g.laplacian(F)) - g.interior(L)).max() / max(1.0, np.abs(L).max())
        if k <= order + 1:
            assert err < 1e-12, (order, k, err)
        else:
            assert err > 1e-8, (order, k, err)


@pytest.mark.parametrize("order", [4, 8, 10])
def test_laplacian_converges_on_a_gaussian(oracle_lib, order):
    errs = []
    for n in (32, 64):
        g = oracle_lib.OracleGrid(oracle_lib.CARTESIAN, n, n, n, order, rmax=5.5)
        X, Y, Z = g.cart()
        r2 = (X - 0.1) ** 2 + (Y + 0.2) ** 2 + (Z - 0.3) ** 2
        F, L = np.exp(-r2), (4.0 * r2 - 6.0) * np.exp(-r2)
        errs.append(np.abs(g.interior(g.laplacian(F)) - g.interior(L)).max())
    rate = np.log2(errs[0] / errs[1])
    assert rate > order - 2, (errs, rate)


def test_classification_map_and_metric(oracle_lib):
    g = oracle_lib.OracleGrid(oracle_lib.CARTESIAN, 10, 8, 6, 8, **CART)
    ng, (N0, N1, N2) = g.NG, g.N
    img = g.bc_images().reshape(g.shape)
    i2, i1, i0 = np.meshgrid(np.arange(g.Nx[2]), np.arange(g.Nx[1]), np.arange(g.Nx[0]),
                             indexing="ij")
    beyond = ((i0 < ng) | (i0 >= ng + N0)).astype(int) + ((i1 < ng) | (i1 >= ng + N1)) + \
        ((i2 < ng) | (i2 >= ng + N2))
    assert np.all((img == -1) == (beyond == 0))
    assert np.all((img == -2) == (beyond == 1))
    assert np.all((img == -4) == (beyond >= 2))
    assert int(np.sum(img == -2)) == 2 * ng * (N1 * N2 + N0 * N2 + N0 * N1)
    # cell-centred cube: x_d = -rmax + (j - NG + 1/2) 2 rmax / N_d
    for d in range(3):
        j = np.arange(g.Nx[d])
        np.testing.assert_allclose(g.xx(d), -6.0 + (j - ng + 0.5) * 12.0 / g.N[d], rtol=0,
                                   atol=1e-14)
    X, Y, Z = g.cart()
    np.testing.assert_array_equal(X[0, 0, :], g.xx(0))
    np.testing.assert_array_equal(Y[0, :, 0], g.xx(1))
    np.testing.assert_array_equal(Z[:, 0, 0], g.xx(2))
    met = g.metric()
    for k in ("a0", "a1", "a2"):
        assert np.all(met[k] == 1.0)
    assert np.all(met["b0"] == 0.0) and np.all(met["b1"] == 0.0)
    assert g.ds_g() == min(g.dxx())


def test_brill_lindquist_stays_exactly_zero(oracle_lib):
    g = oracle_lib.OracleGrid(oracle_lib.CARTESIAN, 8, 8, 8, 8, **CART)
    g.set_punctures([0.5, 0.5], [[0, 0, 1.0], [0, 0, -1.0]], np.zeros((2, 3)), np.zeros((2, 3)))
    _, ssrc = g.sources()
    assert np.all(ssrc == 0.0)
    st, n, hist = g.relax(1.0, 1.0, g.suggest_dt(0.5), 200, 0.0, 50)
    u, v = g.state()
    assert st == 0 and np.all(u == 0.0) and np.all(v == 0.0) and np.all(hist == 0.0)


def test_equal_mass_symmetries(oracle_lib):
    g = oracle_lib.OracleGrid(oracle_lib.CARTESIAN, 12, 10, 8, 8, **CART)
    g.set_punctures([0.5, 0.5], [[0, 0, 1.0], [0, 0, -1.0]], [[0, 0.1, 0], [0, -0.1, 0]],
                    np.zeros((2, 3)))
    st, n, hist = g.relax(1.0, 1.0, g.suggest_dt(0.5), 800, 0.0, 100)
    assert st == 0
    u, _ = g.state()
    img = g.bc_images().reshape(g.shape)
    used = img != -4
    scale = np.abs(u).max()
    assert scale > 0
    # x -> -x: reverse i0
    np.testing.assert_allclose(np.where(used, u[:, :, ::-1], 0), np.where(used, u, 0), rtol=0,
                               atol=1e-13 * scale)
    # (y, z) -> (-y, -z): reverse i1 and i2
    np.testing.assert_allclose(np.where(used, u[::-1, ::-1, :], 0), np.where(used, u, 0),
                               rtol=0, atol=1e-13 * scale)
    # the residual falls
    assert hist[-1] < 0.1 * hist[0]
