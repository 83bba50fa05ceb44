"""Pins of the oracle's puncture sources (paper "Basic equations": Brandt-Bruegmann
punctures, whose Bowen-York extrinsic curvature solves the momentum constraint
analytically, and psi = psi_singular + u).

Checked against what the mathematics fixes rather than the formula itself:
* single-puncture closed forms of the invariant A_ij A^ij derived by hand:
  momentum only  (9 / (2 r^4)) (P^2 + 2 (P.n)^2),
  spin only      (18 / r^6) (S^2 - (S.n)^2);
* A^ij symmetric and trace-free;
* A^ij divergence-free (the momentum constraint with flat conformal metric);
* ADM surface integrals return the input momenta and spins,
  P^i = (1/8pi) oint A^ij n_j dA,  J_i = (1/8pi) oint eps_ijk x^j A^kl n_l dA,
  which fixes the sign of the spin term;
* psi_singular is harmonic away from the punctures and tends to 1 far away;
* the grid source S_src equals (1/8) A_ij A^ij at the grid points.
"""
import numpy as np
import pytest


def _rand_unit(rng, n):
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def test_single_puncture_momentum_invariant(oracle_lib):
    rng = np.random.default_rng(2)
    P = np.array([0.3, -0.7, 0.2])
    pts = _rand_unit(rng, 50) * rng.uniform(0.5, 5.0, size=(50, 1))
    A = oracle_lib.bowen_york([1.0], [0, 0, 0], P, [0, 0, 0], pts)
    r = np.linalg.norm(pts, axis=1)
    n = pts / r[:, None]
    Pn = n @ P
    expect = 9.0 / (2 * r ** 4) * (P @ P + 2 * Pn ** 2)
    np.testing.assert_allclose(np.einsum("kij,kij->k", A, A), expect, rtol=1e-12)


def test_single_puncture_spin_invariant(oracle_lib):
    rng = np.random.default_rng(3)
    S = np.array([-0.1, 0.25, 0.4])
    pts = _rand_unit(rng, 50) * rng.uniform(0.5, 5.0, size=(50, 1))
    A = oracle_lib.bowen_york([1.0], [0, 0, 0], [0, 0, 0], S, pts)
    r = np.linalg.norm(pts, axis=1)
    Sn = (pts / r[:, None]) @ S
    expect = 18.0 / r ** 6 * (S @ S - Sn ** 2)
    np.testing.assert_allclose(np.einsum("kij,kij->k", A, A), expect, rtol=1e-12)


def test_symmetric_trace_free(oracle_lib):
    rng = np.random.default_rng(4)
    m = [0.4, 0.6]
    x = [[0.1, 0.2, 1.0], [-0.3, 0.0, -1.2]]
    P = [[0.1, 0.2, -0.3], [0.0, -0.2, 0.1]]
    S = [[0.0, 0.1, 0.2], [0.3, 0.0, -0.1]]
    pts = rng.uniform(-4, 4, size=(40, 3))
    A = oracle_lib.bowen_york(m, x, P, S, pts)
    scale = np.abs(A).max(axis=(1, 2))
    assert np.all(np.abs(A - A.transpose(0, 2, 1)).max(axis=(1, 2)) < 1e-14 * scale)
    assert np.all(np.abs(np.trace(A, axis1=1, axis2=2)) < 1e-13 * scale)


def test_divergence_free(oracle_lib):
    rng = np.random.default_rng(5)
    m = [0.5, 0.5]
    x = [[0, 0, 1.0], [0, 0, -1.0]]
    P = [[0.1, 0.2, -0.3], [0.0, -0.2, 0.1]]
    S = [[0.0, 0.1, 0.2], [0.3, 0.0, -0.1]]
    pts = rng.uniform(-3, 3, size=(30, 3))
    pts = pts[np.min([np.linalg.norm(pts - np.array(xi), axis=1) for xi in x], axis=0) > 0.8]
    h = 1e-4
    for p in pts:
        div = np.zeros(3)
        scale = np.abs(oracle_lib.bowen_york(m, x, P, S, p[None])[0]).max()
        for j in range(3):
            e = np.zeros(3)
            e[j] = h
            Ap = oracle_lib.bowen_york(m, x, P, S, (p + e)[None])[0]
            Am = oracle_lib.bowen_york(m, x, P, S, (p - e)[None])[0]
            div += (Ap[:, j] - Am[:, j]) / (2 * h)
        assert np.abs(div).max() < 1e-6 * max(scale, 1e-3)


def _sphere_quadrature(R, center, nth=48, nph=96):
    t, w = np.polynomial.legendre.leggauss(nth)  # t = cos(theta)
    ph = (np.arange(nph) + 0.5) * 2 * np.pi / nph
    ct, phg = np.meshgrid(t, ph, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    n = np.stack([st * np.cos(phg), st * np.sin(phg), ct], axis=-1).reshape(-1, 3)
    dA = (np.outer(w, np.full(nph, 2 * np.pi / nph)) * R * R).reshape(-1)
    return center + R * n, n, dA


@pytest.mark.parametrize("R", [3.0, 20.0])
def test_adm_momentum_and_angular_momentum(oracle_lib, R):
    m = [0.5, 0.5]
    x = np.array([[0, 0, 1.0], [0, 0, -1.0]])
    P = np.array([[0.05, 0.1, 0.0], [0.0, -0.1, 0.02]])
    S = np.array([[0.0, 0.1, 0.2], [0.03, 0.0, -0.1]])
    pts, n, dA = _sphere_quadrature(R, np.zeros(3))
    A = oracle_lib.bowen_york(m, x, P, S, pts)
    Pint = np.einsum("kij,kj,k->i", A, n, dA) / (8 * np.pi)
    An = np.einsum("kij,kj->ki", A, n)
    Jint = np.einsum("k,ki->i", dA, np.cross(pts, An)) / (8 * np.pi)
    Ptot = P.sum(axis=0)
    Jtot = (np.cross(x, P) + S).sum(axis=0)
    np.testing.assert_allclose(Pint, Ptot, atol=1e-9)
    np.testing.assert_allclose(Jint, Jtot, atol=1e-9)


def test_grid_sources_match_pointwise_invariant(oracle_lib):
    g = oracle_lib.OracleGrid(0, 16, 12, 4, 8, bscale=1.0)
    m = [0.5, 0.5]
    x = [[0, 0, 1.0], [0, 0, -1.0]]
    P = [[0, 0.1, 0], [0, -0.1, 0]]
    S = [[0, 0, 0.05], [0, 0, -0.02]]
    g.set_punctures(m, x, P, S)
    psi, ssrc = g.sources()
    X, Y, Z = g.cart()
    pts = np.stack([X.reshape(-1), Y.reshape(-1), Z.reshape(-1)], axis=1)
    A = oracle_lib.bowen_york(m, x, P, S, pts)
    np.testing.assert_allclose(ssrc.reshape(-1), np.einsum("kij,kij->k", A, A) / 8, rtol=1e-14)
    # far away psi_singular -> 1 + M/(2r)
    r = np.sqrt(X ** 2 + Y ** 2 + Z ** 2)
    far = r > 1e4
    np.testing.assert_allclose(psi[far], 1 + 1.0 / (2 * r[far]), rtol=1e-8)


def test_psi_singular_is_harmonic(oracle_lib):
    # lap(psi_s) = 0 away from the punctures, at the stencil's order
    errs = []
    for N in (24, 48):
        g = oracle_lib.OracleGrid(0, N, N, N, 8, amax=30.0, sinhwaa=0.3, bscale=1.0)
        g.set_punctures([0.5, 0.5], [[0, 0, 1.0], [0, 0, -1.0]], np.zeros((2, 3)), np.zeros((2, 3)))
        psi, _ = g.sources()
        L = g.interior(g.laplacian(psi))
        x0 = g.xx(0)[g.NG:g.NG + N]
        x1 = g.xx(1)[g.NG:g.NG + N]
        mask = np.broadcast_to(((np.sin(x1) > 0.5)[:, None] & ((x0 > 0.3) & (x0 < 0.8))[None, :])[None],
                               L.shape)
        errs.append(np.abs(L[mask]).max())
    assert np.log2(errs[0] / errs[1]) > 6.0
