"""Pins for the FP64 importance-network oracle: BF16 rounding against torch's
conversion, gradients against central finite differences, Adam against its
closed-form first step, and training that fits a known target."""
import numpy as np
import pytest
import torch

from oracle import mlp


def test_bf16_round_matches_torch_conversion():
    rng = np.random.default_rng(0)
    a = np.concatenate([rng.normal(size=5000) * 10.0 ** rng.integers(-20, 20, 5000),
                        [0.0, -0.0, 1.0, -1.0, 3.0e38, 1e-40, 0.5 + 2 ** -9, 0.5 + 3 * 2 ** -9]])
    ours = mlp.bf16_round(a)
    ref = torch.tensor(a.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(ours, ref)


def _data(n=64, seed=1):
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1, 1, (n, 4))
    t = np.sin(2 * x[:, 0]) + 0.5 * x[:, 3] ** 2
    w = rng.uniform(0.5, 2.0, n)
    return x, t, w


def test_gradients_match_central_differences():
    p = mlp.init_params(3)
    p.b1 = np.random.default_rng(4).normal(0, 0.1, 64)
    p.b2 = np.random.default_rng(5).normal(0, 0.1, 64)
    p.b3 = 0.3
    x, t, w = _data()
    y, cache = mlp.forward(p, x, rounding=False)
    g = mlp.backward(p, cache, y, t, w).flat()
    th = p.flat()
    rng = np.random.default_rng(6)
    idx = np.concatenate([rng.choice(mlp.N_PARAMS, 200, replace=False), [mlp.N_PARAMS - 1, 0, 300, 4500]])
    h = 1e-6
    for i in idx:
        tp, tm = th.copy(), th.copy()
        tp[i] += h
        tm[i] -= h
        lp = mlp.loss(mlp.forward(mlp.Params.from_flat(tp), x, False)[0], t, w)
        lm = mlp.loss(mlp.forward(mlp.Params.from_flat(tm), x, False)[0], t, w)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(fd)) + 1e-9, (i, fd, g[i])


def test_silu_grad_is_derivative():
    z = np.linspace(-8, 8, 101)
    h = 1e-6
    np.testing.assert_allclose(mlp.silu_grad(z), (mlp.silu(z + h) - mlp.silu(z - h)) / (2 * h), atol=1e-8)


def test_rounded_forward_differs_from_exact_only_by_bf16():
    p = mlp.init_params(7)
    x, _, _ = _data(256, 8)
    y_r, _ = mlp.forward(p, x, True)
    y_e, _ = mlp.forward(p, x, False)
    # BF16 keeps 8 significant bits: the network output moves by well under 5 %
    assert np.max(np.abs(y_r - y_e)) < 0.05 * (1 + np.max(np.abs(y_e)))
    assert not np.array_equal(y_r, y_e)


def test_adam_first_step_is_signed_lr():
    """After one step Adam moves every parameter with a nonzero gradient by
    lr * g / (|g| + eps) (bias-corrected moments equal g and g^2)."""
    p = mlp.init_params(9)
    x, t, w = _data()
    y, cache = mlp.forward(p, x)
    g = mlp.backward(p, cache, y, t, w)
    q = mlp.Adam(lr=1e-3).step(p, g)
    d = q.flat() - p.flat()
    gf = g.flat()
    np.testing.assert_allclose(d, -1e-3 * gf / (np.abs(gf) + 1e-8), rtol=1e-9, atol=1e-15)


def test_training_fits_a_linear_log_importance():
    """ln I linear in depth (the pure-absorber shape) is learned to a small
    residual."""
    rng = np.random.default_rng(10)
    n = 400
    xs = rng.uniform(0, 1, n)
    x = np.stack([xs, rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), rng.uniform(0, 1, n)], axis=1)
    t = 6.0 * xs - 3.0
    w = np.ones(n)
    p, curve = mlp.train(mlp.init_params(11), x, t, w, steps=600, lr=1e-2)
    assert curve[-1] < 0.01 * curve[0]
    y, _ = mlp.forward(p, x)
    assert np.sqrt(np.mean((y - t) ** 2)) < 0.15
