"""Pin of the numpy MLP oracle: its chain-rule gradient must equal central
finite differences of its own loss (brute force on a tiny network)."""
import numpy as np

from oracle import mlp


def test_oracle_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    width = 8
    n = mlp.N_FEAT * width + width + width * width + width + width + 1
    p = rng.normal(scale=0.5, size=n)
    x = rng.normal(size=(5, mlp.N_FEAT))
    t = rng.normal(size=5)
    loss, g = mlp.loss_and_grad(p, width, x, t)
    h = 1e-6
    fd = np.zeros(n)
    for i in range(n):
        pp = p.copy(); pp[i] += h
        pm = p.copy(); pm[i] -= h
        fd[i] = (mlp.loss_and_grad(pp, width, x, t)[0] - mlp.loss_and_grad(pm, width, x, t)[0]) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-8)
    assert loss > 0


def test_gelu_known_values():
    # GELU(0) = 0, GELU(z) -> z for large z, GELU(-z) = GELU(z) - z
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    np.testing.assert_allclose(mlp.gelu(np.array([8.0])), [8.0], rtol=1e-12)
    z = np.array([0.3, 1.7, 2.5])
    np.testing.assert_allclose(mlp.gelu(-z), mlp.gelu(z) - z, rtol=1e-14, atol=1e-15)
