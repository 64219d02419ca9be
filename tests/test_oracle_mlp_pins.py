"""Pins of the FP64 MLP oracle: gradients against central finite differences,
the Adam step against its closed form, and the parameter count of the
6 -> 4 x 128 -> 4 warm-start network."""
import numpy as np

from oracle import mlp


def test_parameter_count():
    p = mlp.init_params(6, 128, 4, 4, seed=0)
    assert sum(W.size + b.size for W, b in p) == 50948


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(1)
    p = mlp.init_params(6, 16, 3, 4, seed=2)
    x = rng.normal(size=(32, 6))
    y = rng.normal(size=(32, 4))
    loss, grads = mlp.loss_and_grads(p, x, y)
    flat = mlp.flatten(p)
    gflat = np.concatenate([np.concatenate([gW.ravel(), gb.ravel()]) for gW, gb in grads])
    eps = 1e-6
    idx = rng.choice(len(flat), 200, replace=False)
    for i in idx:
        fp = flat.copy()
        fp[i] += eps
        fm = flat.copy()
        fm[i] -= eps
        lp = mlp.loss_and_grads(mlp.unflatten(fp, 6, 16, 3, 4), x, y)[0]
        lm = mlp.loss_and_grads(mlp.unflatten(fm, 6, 16, 3, 4), x, y)[0]
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - gflat[i]) <= 1e-6 * max(1e-3, abs(gflat[i])) + 1e-10


def test_silu_derivative():
    z = np.linspace(-8, 8, 101)
    fd = (mlp.silu(z + 1e-6) - mlp.silu(z - 1e-6)) / 2e-6
    np.testing.assert_allclose(mlp.dsilu(z), fd, rtol=1e-7, atol=1e-10)


def test_adam_first_step_closed_form():
    """First Adam step: m_hat = g, v_hat = g^2, so every parameter moves by
    -lr g / (|g| + eps) ~ -lr sign(g)."""
    rng = np.random.default_rng(3)
    p = [(rng.normal(size=(3, 2)), rng.normal(size=2))]
    g = [(rng.normal(size=(3, 2)), rng.normal(size=2))]
    z = [(np.zeros((3, 2)), np.zeros(2))]
    new, m, v = mlp.adam_step(p, g, z, z, t=1, lr=1e-3)
    for (W, b), (W0, b0), (gW, gb) in zip(new, p, g):
        np.testing.assert_allclose(W - W0, -1e-3 * gW / (np.abs(gW) + 1e-8), rtol=1e-10)
        np.testing.assert_allclose(b - b0, -1e-3 * gb / (np.abs(gb) + 1e-8), rtol=1e-10)


def test_loss_decreases_under_training():
    rng = np.random.default_rng(4)
    x = rng.normal(size=(256, 6))
    y = np.stack([np.sin(x[:, 0]), x[:, 1] * x[:, 2], np.tanh(x[:, 3]), x[:, 4] - x[:, 5]], axis=1)
    p = mlp.init_params(6, 32, 2, 4, seed=5)
    m = [(np.zeros_like(W), np.zeros_like(b)) for W, b in p]
    v = [(np.zeros_like(W), np.zeros_like(b)) for W, b in p]
    l0 = mlp.loss_and_grads(p, x, y)[0]
    for t in range(1, 301):
        loss, g = mlp.loss_and_grads(p, x, y)
        p, m, v = mlp.adam_step(p, g, m, v, t, lr=3e-3)
    assert loss < 0.2 * l0
