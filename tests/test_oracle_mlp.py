"""Pins of the FP64 reference network: GELU identities and finite differences."""
import numpy as np

from oracle import mlp


def test_gelu_identities():
    z = np.linspace(-6, 6, 25)
    assert abs(mlp.gelu(np.array([0.0]))[0]) == 0.0
    assert np.allclose(mlp.gelu(z) - mlp.gelu(-z), z, atol=1e-15)          # GELU(z) - GELU(-z) = z
    assert abs(mlp.gelu(np.array([40.0]))[0] - 40.0) < 1e-12
    h = 1e-6
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    assert np.allclose(fd, mlp.gelu_grad(z), atol=1e-8)


def test_backward_matches_central_differences():
    rng = np.random.default_rng(3)
    n_in, width, depth = 5, 16, 2
    p = mlp.init_params(n_in, width, depth, rng) + rng.normal(0, 0.05, mlp.param_count(n_in, width, depth))
    x = rng.normal(0, 1, (7, mlp.in_pad(n_in)))
    t = rng.normal(0, 1, 7)
    _, g = mlp.loss_and_grad(p, x, t, n_in, width, depth)
    h = 1e-6
    for i in rng.choice(len(p), 40, replace=False):
        e = np.zeros_like(p)
        e[i] = h
        fd = (mlp.loss_and_grad(p + e, x, t, n_in, width, depth)[0]
              - mlp.loss_and_grad(p - e, x, t, n_in, width, depth)[0]) / (2 * h)
        assert abs(fd - g[i]) < 1e-7 * max(1.0, abs(g[i]))


def test_features_are_unit_vectors():
    from oracle import philox
    a = philox.sample_angles(1, 0, 9, 4)
    x = mlp.features(a, [0.0, 2.0])
    assert x.shape == (18, 16)
    n = x[:, :12].reshape(18, 4, 3)
    assert np.allclose((n * n).sum(axis=2), 1.0)
    assert np.allclose(x[:9, 12], np.log(0.05)) and np.allclose(x[9:, 12], np.log(2.05))
    assert np.all(x[:, 13:] == 0)


def test_adam_first_step_moves_by_lr():
    p, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    g = np.array([1.0, -2.0, 0.5])
    p1, _, _ = mlp.adam(p, m, v, g, 1, 0.01)
    assert np.allclose(p1, -0.01 * np.sign(g), rtol=1e-6)     # bias-corrected first step is lr*sign(g)


def test_cv_beta_recovers_linear_relation():
    rng = np.random.default_rng(0)
    g = rng.normal(0, 1, (3, 500))
    phi = 0.7 * g + 0.2
    assert np.allclose(mlp.cv_beta(phi, g), 0.7)
