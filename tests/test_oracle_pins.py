"""Pins of three oracle functions against facts fixed outside the oracle.

* Grid L2 norm (the stop test's norm, "Data transfer" subsection of the
  paper's Sec. 4: the grid L2 norm of the Hamiltonian-constraint violations):
  with Brill-Lindquist sources (no momentum, no spin, so the source term is
  exactly zero) and u = r^p on a Spherical grid, H = lap(r^p) = p (p+1) r^(p-2)
  exactly (the centred stencils are exact on these polynomials), so the norm
  must equal the root mean square of that closed form over the interior
  points.
* SinhSymTP radiation condition: at the outer points the slope must be
  -c (f/r + (df/dxx0) / (dr/dxx0)); a one-sided difference of order p is exact
  on polynomials of degree p in xx0, so for such fields the oracle must match
  the closed form with dr/dxx0 taken from a numerical derivative of the
  coordinate map (not from the oracle's own expression).
* Eq. (4) source factor and exponent: a single puncture of mass m with a small
  momentum P (no spin) has u = O(P^2), and to that order u solves the linear
  equation lap u = -(1/8) |A|^2 psi0^-7, psi0 = 1 + m/(2r), with
  |A|^2 = (9 P^2 / (2 r^4)) (1 + 2 cos^2 theta) for the Bowen-York momentum
  term. Its l = 0 and l = 2 parts are radial ODEs; their solutions, regular at
  the origin and with the radiation condition's steady state u' + u/R = 0 at
  the outer radius R, are written below with Green's functions and evaluated
  by quadrature. The oracle relaxed to convergence must reproduce them, with
  the error falling under refinement.

Each helper returns error measures, so that ``test_oracle_mutations.py`` can
run the same checks on copies of the oracle with a planted mistake.
"""
from __future__ import annotations

import numpy as np
import pytest
from scipy import integrate


# --- grid L2 norm ---------------------------------------------------------

def grid_norm_errors(orc) -> list[float]:
    g = orc.OracleGrid(orc.SPHERICAL, 20, 8, 4, 8, rmax=3.0)
    # Brill-Lindquist: P = S = 0, so the source term vanishes identically
    g.set_punctures([0.5], [[0.3, -0.2, 0.4]], [[0, 0, 0]], [[0, 0, 0]])
    ng, (N0, N1, N2) = g.NG, g.N
    x0 = g.xx(0)          # padded; inner ghosts have x0 < 0 and even powers match their images
    errs = []
    for p in (2, 4):
        U = np.broadcast_to((x0 ** p)[None, None, :], g.shape).copy()
        got = g.residual(U)
        r = x0[ng:ng + N0]
        H = p * (p + 1) * r ** (p - 2)
        # every (i1, i2) row holds the same values: the mean over N0*N1*N2
        # points is the mean over one row
        want = np.sqrt(np.sum(H ** 2) * N1 * N2 / (N0 * N1 * N2))
        errs.append(abs(got - want) / want)
    return errs


def check_grid_norm(orc) -> None:
    errs = grid_norm_errors(orc)
    assert max(errs) < 1e-12, errs


def test_grid_l2_norm_is_rms_over_interior_points(oracle_lib):
    check_grid_norm(oracle_lib)


# --- SinhSymTP radiation condition ------------------------------------------

SINHSYMTP_MILD = dict(amax=3.0, sinhwaa=0.4, bscale=1.0)


def _drdx0_numeric(g, x0: float, x1: float) -> float:
    """d|x|/dxx0 at fixed (xx1, xx2) from the coordinate map, sixth-order
    centred difference."""
    h = 1e-3
    f = lambda t: float(np.linalg.norm(g.to_cart(t, x1, 0.3)))  # noqa: E731
    return (-f(x0 - 3 * h) + 9 * f(x0 - 2 * h) - 45 * f(x0 - h) + 45 * f(x0 + h)
            - 9 * f(x0 + 2 * h) + f(x0 + 3 * h)) / (60 * h)


def sinhsymtp_bc_errors(orc, order: int = 2):
    """(max error for degrees <= order, error at degree order + 1), relative."""
    g = orc.OracleGrid(orc.SINHSYMTP, 16, 8, 4, 8, **SINHSYMTP_MILD)
    g.set_bc_order(order)
    ng, (N0, N1, N2) = g.NG, g.N
    x0 = g.xx(0)
    x1 = g.xx(1)
    xo = x0[ng + N0:]
    X, Y, Z = g.cart()
    r = np.sqrt(X ** 2 + Y ** 2 + Z ** 2)[ng:ng + N2, ng:ng + N1, ng + N0:]
    met = g.metric()
    c = met["dsmin"][ng:ng + N1, ng + N0:] / g.ds_g()
    drdx = np.array([[_drdx0_numeric(g, a, b) for a in xo] for b in x1[ng:ng + N1]])
    exact_err, beyond_err = 0.0, 0.0
    for deg in range(order + 2):
        fx = np.polynomial.Polynomial(np.arange(1, deg + 2, dtype=float) / (deg + 1))
        f = np.broadcast_to(fx(x0)[None, None, :], g.shape).copy()
        ku, _ = g.rhs(0.0, 1.0, f, np.zeros(g.shape))
        got = ku[ng:ng + N2, ng:ng + N1, ng + N0:]
        want = -c[None] * (fx(xo)[None, None] / r + fx.deriv()(xo)[None, None] / drdx[None])
        err = float(np.abs(got - want).max() / np.abs(want).max())
        if deg <= order:
            exact_err = max(exact_err, err)
        else:
            beyond_err = err
    return exact_err, beyond_err


def check_sinhsymtp_bc(orc, order: int = 2) -> None:
    exact, beyond = sinhsymtp_bc_errors(orc, order)
    assert exact < 1e-10, exact
    assert beyond > 1e-8, beyond


@pytest.mark.parametrize("order", [2, 4])
def test_sinhsymtp_radiation_condition_exact_on_polynomials(oracle_lib, order):
    check_sinhsymtp_bc(oracle_lib, order)


# --- SinhCylindrical radiation condition (rho face and both z faces) -------

SINHCYL_MILD = dict(amax=3.0, sinhwaa=0.4)


def _drdx_numeric(g, x0: float, x1: float, d: int) -> float:
    """d|x|/dxx_d at fixed other coordinates from the coordinate map,
    sixth-order centred difference."""
    h = 1e-3

    def f(t):
        a = [x0, x1, 0.3]
        a[d] = t
        return float(np.linalg.norm(g.to_cart(*a)))

    t = (x0, x1)[d]
    return (-f(t - 3 * h) + 9 * f(t - 2 * h) - 45 * f(t - h) + 45 * f(t + h)
            - 9 * f(t + 2 * h) + f(t + 3 * h)) / (60 * h)


def sinhcylindrical_bc_errors(orc, order: int = 2):
    """(max error for degrees <= order, smallest error at degree order + 1),
    relative, over the rho face (fields polynomial in xx0) and the z faces
    with their corners (fields polynomial in xx1)."""
    g = orc.OracleGrid(orc.SINHCYLINDRICAL, 12, 10, 4, 8, **SINHCYL_MILD)
    g.set_bc_order(order)
    ng, (N0, N1, N2) = g.NG, g.N
    x0, x1 = g.xx(0), g.xx(1)
    X, Y, Z = g.cart()
    r = np.sqrt(X ** 2 + Y ** 2 + Z ** 2)
    c = g.metric()["dsmin"] / g.ds_g()          # (Nx1, Nx0) plane
    zrows = list(range(ng)) + list(range(ng + N1, N1 + 2 * ng))

    def along_z(b, a):   # the reading: along xx1 where |z| >= rho
        p = g.to_cart(x0[a], x1[b], 0.0)
        return abs(p[2]) >= abs(p[0])

    zpts = [(b, a) for b in zrows for a in range(ng, N0 + 2 * ng)]
    faces = [
        # rho face (interior rows, outer columns) and the z-face points nearer
        # to it (rho > |z|): derivative along xx0
        (0, [(b, a) for b in range(ng, ng + N1) for a in range(ng + N0, N0 + 2 * ng)] +
            [q for q in zpts if not along_z(*q)]),
        # z-face points with |z| >= rho: derivative along xx1
        (1, [q for q in zpts if along_z(*q)]),
    ]
    assert len(faces[1][1]) > 0 and len(faces[0][1]) > N1 * ng
    exact_err, beyond_err = 0.0, np.inf
    for d, pts in faces:
        drdx = np.array([_drdx_numeric(g, x0[a], x1[b], d) for b, a in pts])
        ib = np.array([b for b, _ in pts])
        ia = np.array([a for _, a in pts])
        for deg in range(order + 2):
            fx = np.polynomial.Polynomial(np.arange(1, deg + 2, dtype=float) / (deg + 1))
            prof = fx(x0) if d == 0 else fx(x1)
            f = np.broadcast_to(prof[None, None, :] if d == 0 else prof[None, :, None],
                                g.shape).copy()
            ku, _ = g.rhs(0.0, 1.0, f, np.zeros(g.shape))
            got = ku[ng:ng + N2][:, ib, ia]
            t = x0[ia] if d == 0 else x1[ib]
            want = -c[ib, ia][None] * (fx(t)[None] / r[ng:ng + N2][:, ib, ia] +
                                       fx.deriv()(t)[None] / drdx[None])
            err = float(np.abs(got - want).max() / np.abs(want).max())
            if deg <= order:
                exact_err = max(exact_err, err)
            else:
                beyond_err = min(beyond_err, err)
    return exact_err, beyond_err


def check_sinhcylindrical_bc(orc, order: int = 2) -> None:
    exact, beyond = sinhcylindrical_bc_errors(orc, order)
    assert exact < 1e-10, exact
    assert beyond > 1e-8, beyond


@pytest.mark.parametrize("order", [2, 4])
def test_sinhcylindrical_radiation_condition_exact_on_polynomials(oracle_lib, order):
    check_sinhcylindrical_bc(oracle_lib, order)


def cartesian_bc_errors(orc, order: int = 2):
    """(max error for degrees <= order, smallest error at degree order + 1),
    relative, over the six faces of a Cartesian grid: on the two faces normal
    to x_d the field is a polynomial in x_d, the condition's one-sided
    difference runs along x_d toward the interior and d r / d x_d is taken
    from the coordinate map numerically."""
    g = orc.OracleGrid(orc.CARTESIAN, 10, 8, 6, 8, rmax=3.0)
    g.set_bc_order(order)
    ng, N = g.NG, g.N
    X, Y, Z = g.cart()
    r = np.sqrt(X ** 2 + Y ** 2 + Z ** 2)
    img = g.bc_images()
    c = g.metric()["dsmin"] / g.ds_g()   # uniform on this grid
    exact_err, beyond_err = 0.0, np.inf
    h = 1e-3
    for d in range(3):
        xs = g.xx(d)
        idx = np.argwhere(img.reshape(g.shape) == -2)   # (i2, i1, i0)
        # face points beyond a face normal to x_d
        pts = np.array([q for q in idx
                        if q[2 - d] < ng or q[2 - d] >= ng + N[d]])
        assert len(pts) == 2 * ng * int(np.prod(N)) // N[d]
        i2, i1, i0 = pts[:, 0], pts[:, 1], pts[:, 2]
        xd = (X, Y, Z)[d][i2, i1, i0]
        # d |x| / d x_d from the map at each point (sixth-order difference)
        base = np.stack([X[i2, i1, i0], Y[i2, i1, i0], Z[i2, i1, i0]], axis=1)

        def rad(t):
            p = base.copy()
            p[:, d] = t
            return np.array([np.linalg.norm(g.to_cart(*q)) for q in p])

        drdx = (-rad(xd - 3 * h) + 9 * rad(xd - 2 * h) - 45 * rad(xd - h) + 45 * rad(xd + h)
                - 9 * rad(xd + 2 * h) + rad(xd + 3 * h)) / (60 * h)
        for deg in range(order + 2):
            fx = np.polynomial.Polynomial(np.arange(1, deg + 2, dtype=float) / (deg + 1))
            shape = [1, 1, 1]
            shape[2 - d] = len(xs)
            f = np.broadcast_to(fx(xs).reshape(shape), g.shape).copy()
            ku, _ = g.rhs(0.0, 1.0, f, np.zeros(g.shape))
            got = ku[i2, i1, i0]
            want = -c[i1, i0] * (fx(xd) / r[i2, i1, i0] + fx.deriv()(xd) / drdx)
            err = float(np.abs(got - want).max() / np.abs(want).max())
            if deg <= order:
                exact_err = max(exact_err, err)
            else:
                beyond_err = min(beyond_err, err)
    return exact_err, beyond_err


def check_cartesian_bc(orc, order: int = 2) -> None:
    exact, beyond = cartesian_bc_errors(orc, order)
    assert exact < 1e-10, exact
    assert beyond > 1e-8, beyond


@pytest.mark.parametrize("order", [2, 4])
def test_cartesian_radiation_condition_exact_on_polynomials(oracle_lib, order):
    check_cartesian_bc(oracle_lib, order)


# --- Eq. (4): source factor and exponent ------------------------------------

def boosted_puncture_u(m: float, P: float, R: float, r: np.ndarray, cos_t: np.ndarray):
    """O(P^2) solution u(r, theta) for one puncture of mass m at the origin with
    momentum P along z, on 0 <= r <= R with u' + u/R = 0 at R.

    lap u = g0(r) + g2(r) P2(cos theta), with
    g0 = -(1/8)(9 P^2/(2 r^4))(5/3) psi0^-7 and g2 = -(1/8)(9 P^2/(2 r^4))(4/3) psi0^-7
    (1 + 2 cos^2 = 5/3 + (4/3) P2).
    l = 0: (r^2 u0')' = r^2 g0, so u0' = Q(r)/r^2 with Q = int_0^r s^2 g0 ds and
    u0(r) = -Q(R)/R - int_r^R Q(s)/s^2 ds.
    l = 2: (r^2 u2')' - 6 u2 = r^2 g2; homogeneous solutions y1 = r^2 (regular)
    and y2 = r^-3 + (2/(3 R^5)) r^2 (meets the outer condition);
    r^2 (y1 y2' - y1' y2) = -5, so
    u2(r) = -(1/5)[y2(r) int_0^r y1 s^2 g2 ds + y1(r) int_r^R y2 s^2 g2 ds]."""
    psi0 = lambda s: 1.0 + m / (2.0 * s)                                  # noqa: E731
    amp = 9.0 * P * P / 2.0 / 8.0
    g0 = lambda s: -amp * (5.0 / 3.0) * s ** -4 * psi0(s) ** -7          # noqa: E731
    g2 = lambda s: -amp * (4.0 / 3.0) * s ** -4 * psi0(s) ** -7          # noqa: E731
    kw = dict(epsabs=0.0, epsrel=1e-12, limit=200)
    Q = lambda x: integrate.quad(lambda s: s * s * g0(s), 0.0, x, **kw)[0]  # noqa: E731
    QR = Q(R)
    beta = 2.0 / (3.0 * R ** 5)
    y1 = lambda s: s * s                                                  # noqa: E731
    y2 = lambda s: s ** -3 + beta * s * s                                 # noqa: E731
    radial = {}
    for x in np.unique(r):
        u0 = -QR / R - integrate.quad(lambda s: Q(s) / s ** 2, x, R, **kw)[0]
        a = integrate.quad(lambda s: y1(s) * s * s * g2(s), 0.0, x, **kw)[0]
        b = integrate.quad(lambda s: y2(s) * s * s * g2(s), x, R, **kw)[0]
        radial[x] = (u0, -(y2(x) * a + y1(x) * b) / 5.0)
    u0 = np.array([radial[x][0] for x in r.ravel()]).reshape(r.shape)
    u2 = np.array([radial[x][1] for x in r.ravel()]).reshape(r.shape)
    return u0 + u2 * 0.5 * (3.0 * cos_t ** 2 - 1.0)


def boosted_puncture_errors(orc, resolutions=((48, 12), (96, 24))) -> list[float]:
    """max|u_oracle - u_ref| / max|u_ref| over the interior after relaxing to
    convergence, per resolution (Spherical, R = 12, 8th order)."""
    m, P, R = 1.0, 0.01, 12.0
    errs = []
    for N0, N1 in resolutions:
        g = orc.OracleGrid(orc.SPHERICAL, N0, N1, 2, 8, rmax=R)
        g.set_punctures([m], [[0, 0, 0]], [[0, 0, P]], [[0, 0, 0]])
        r0 = g.residual()
        st, steps, hist = g.relax(2.0, 1.0, g.suggest_dt(0.5), 40000, 1e-10 * r0, 100)
        if st != 0:
            errs.append(float("inf"))
            continue
        u, _ = g.state()
        ui = g.interior(u)
        X, Y, Z = g.cart()
        Rc = np.sqrt(X ** 2 + Y ** 2 + Z ** 2)
        rr, ct = g.interior(Rc), g.interior(Z / Rc)
        uref = boosted_puncture_u(m, P, R, rr, ct)
        errs.append(float(np.abs(ui - uref).max() / np.abs(uref).max()))
    return errs


def check_boosted_puncture(orc) -> None:
    e_coarse, e_fine = boosted_puncture_errors(orc)
    assert e_coarse < 5e-3, (e_coarse, e_fine)
    assert e_fine < 5e-4, (e_coarse, e_fine)
    assert e_fine < e_coarse / 4, (e_coarse, e_fine)


def test_relaxed_u_matches_perturbative_boosted_puncture(oracle_lib):
    check_boosted_puncture(oracle_lib)
