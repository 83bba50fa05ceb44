"""Pins of the oracle's outer radiation condition, k_f = -c (f/r + d_r f), with
the radial derivative taken along xx0 by a one-sided difference of order 2
(default) or 4.

* Exactness: a one-sided difference of order p through p + 1 points is exact
  on polynomials of degree p in xx0. On a Spherical grid (r = xx0) and on a
  SinhSpherical grid (r = A(xx0), d_r = d_xx0 / A') the outer-point slopes of
  a field that is a polynomial in xx0 must equal the closed form -c (f/r +
  f'/A') to rounding for degree <= order, and must not for degree order + 1.
* Convergence: on a smooth non-polynomial field the error of the outer slopes
  falls as h^order under refinement.
"""
import numpy as np
import pytest

SSPH_MILD = dict(amax=3.0, sinhwaa=0.4)


def _outer_slopes(g, f, kappa=1.0):
    """ku at the outer points (padded layout) for u = f, v = 0."""
    ku, _ = g.rhs(0.0, kappa, f, np.zeros(g.shape))
    ng, (N0, N1, N2) = g.NG, g.N
    return ku[ng:ng + N2, ng:ng + N1, ng + N0:]


def _exact(g, fx, dfx, kappa=1.0):
    """-c (f/r + f'(xx0) / (dr/dxx0)) at the outer points, with c = kappa
    ds_min / ds_g from the oracle's own metric table."""
    ng, (N0, N1, N2) = g.NG, g.N
    x0 = g.xx(0)[ng + N0:]
    X, Y, Z = g.cart()
    r = np.sqrt(X ** 2 + Y ** 2 + Z ** 2)[ng:ng + N2, ng:ng + N1, ng + N0:]
    met = g.metric()
    c = kappa * met["dsmin"][ng:ng + N1, ng + N0:] / g.ds_g()
    drdx = 1.0 / np.sqrt(met["a0"][ng:ng + N1, ng + N0:])   # h0 = dr/dxx0 on these grids
    return -c[None] * (fx(x0)[None, None] / r + dfx(x0)[None, None] / drdx[None])


def _field(g, fx):
    x0 = g.xx(0)
    return np.broadcast_to(fx(x0)[None, None, :], g.shape).copy()


GRIDS = [(1, dict(rmax=2.0)), (2, SSPH_MILD)]


@pytest.mark.parametrize("coords,kw", GRIDS)
@pytest.mark.parametrize("order", [2, 4])
def test_one_sided_difference_is_exact_on_polynomials(oracle_lib, coords, kw, order):
    g = oracle_lib.OracleGrid(coords, 24, 8, 4, 8, **kw)
    g.set_bc_order(order)
    for deg in range(order + 2):
        coef = np.arange(1, deg + 2, dtype=float) / (deg + 1)
        fx = np.polynomial.Polynomial(coef)
        got = _outer_slopes(g, _field(g, fx))
        want = _exact(g, fx, fx.deriv())
        err = np.abs(got - want).max() / np.abs(want).max()
        if deg <= order:
            assert err < 1e-11, (order, deg, err)
        else:
            assert err > 1e-8, (order, deg, err)


@pytest.mark.parametrize("coords,kw", GRIDS)
@pytest.mark.parametrize("order", [2, 4])
def test_one_sided_difference_converges_at_its_order(oracle_lib, coords, kw, order):
    fx = lambda x: np.exp(-0.7 * x) * np.cos(1.3 * x)          # noqa: E731
    dfx = lambda x: -np.exp(-0.7 * x) * (0.7 * np.cos(1.3 * x) + 1.3 * np.sin(1.3 * x))  # noqa: E731
    errs = []
    for n in (16, 32, 64):
        g = oracle_lib.OracleGrid(coords, n, 8, 4, 8, **kw)
        g.set_bc_order(order)
        got = _outer_slopes(g, _field(g, fx))
        want = _exact(g, fx, dfx)
        # the outer points move with the grid: compare the difference error
        # scaled by the local derivative term
        errs.append(np.abs(got - want).max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > order - 0.6), (order, errs, rates)


def test_bc_order_rejections(oracle_lib):
    g = oracle_lib.OracleGrid(1, 24, 8, 4, 8, rmax=2.0)
    with pytest.raises(ValueError):
        g.set_bc_order(3)
    small = oracle_lib.OracleGrid(1, 3, 4, 2, 4, rmax=2.0)
    with pytest.raises(ValueError):
        small.set_bc_order(4)        # the difference would reach an inner ghost
    small.set_bc_order(2)
