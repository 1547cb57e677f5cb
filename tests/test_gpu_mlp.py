"""GPU parity of the importance network (inference, gradient, Adam training)
against the FP64 oracle with the same BF16 rounding points, through the C ABI.

Bars (FP32 arithmetic against FP64 with identical rounding points):
  * forward: 99 % of outputs within 2e-5 (1 + |y|), every output within
    1e-2 (1 + |y|) -- the loose bound covers the rare sample where FP32 and
    FP64 round one hidden activation to different BF16 neighbours;
  * gradient: every component within 2e-3 of the largest component of its
    parameter block, 99 % within 2e-4 of it; loss within 1e-5 relative;
  * training: the loss curve of 10 Adam steps within 1e-4 relative, 99 % of
    the parameters within 1e-5 absolute at the end.
"""
import sys

import numpy as np
import pytest

from oracle import mlp
from paper_2403_12345_amd import mc

pytestmark = pytest.mark.gpu

BLOCKS = {"W1": (0, 256), "b1": (256, 320), "W2": (320, 4416), "b2": (4416, 4480), "w3": (4480, 4544),
          "b3": (4544, 4545)}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    return torch


@pytest.fixture(scope="module")
def ctx(torch_cuda):
    c = mc.mc_create(0)
    yield c
    mc.mc_destroy(c)


def _params(seed):
    p = mlp.init_params(seed)
    rng = np.random.default_rng(seed + 100)
    p.b1 = rng.normal(0, 0.3, 64)
    p.b2 = rng.normal(0, 0.3, 64)
    p.b3 = 0.4
    # the kernels take FP32 parameters: the oracle sees the same FP32 values
    return mlp.Params.from_flat(p.flat().astype(np.float32).astype(np.float64))


def _features(n, seed):
    rng = np.random.default_rng(seed)
    f = np.stack([rng.uniform(0, 1, n), rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), rng.uniform(0, 1, n)], 1)
    return f.astype(np.float32)


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


@pytest.mark.parametrize("n", [1, 63, 64, 255, 256, 1000, 70_001])
def test_forward_matches_oracle(ctx, torch_cuda, n):
    torch = torch_cuda
    _say(f"mlp forward n={n}")
    p = _params(1)
    mc.mc_mlp_set(ctx, p.flat())
    f = _features(n, n)
    X = _dev(torch, f)
    Y = torch.full((n,), float("nan"), dtype=torch.float32, device="cuda")
    mc.mc_mlp_forward(ctx, n, X, Y)
    torch.cuda.synchronize()
    got = Y.cpu().numpy().astype(np.float64)
    ref, _ = mlp.forward(p, f.astype(np.float64))
    err = np.abs(got - ref) / (1.0 + np.abs(ref))
    assert np.all(np.isfinite(got))
    assert np.max(err) <= 1e-2, np.max(err)
    assert np.mean(err <= 2e-5) >= 0.99, np.sort(err)[-10:]


def test_forward_is_deterministic_and_zero_length_is_a_no_op(ctx, torch_cuda):
    torch = torch_cuda
    mc.mc_mlp_set(ctx, _params(2).flat())
    X = _dev(torch, _features(5000, 3))
    a = torch.empty(5000, dtype=torch.float32, device="cuda")
    b = torch.empty(5000, dtype=torch.float32, device="cuda")
    mc.mc_mlp_forward(ctx, 5000, X, a)
    mc.mc_mlp_forward(ctx, 5000, X, b)
    mc.mc_mlp_forward(ctx, 0, X, b)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_get_returns_what_set_loaded(ctx, torch_cuda):
    v = _params(3).flat().astype(np.float32)
    mc.mc_mlp_set(ctx, v)
    assert np.array_equal(mc.mc_mlp_get(ctx), v)
    bad = v.copy()
    bad[17] = np.nan
    with pytest.raises(mc.MCError):
        mc.mc_mlp_set(ctx, bad)


def _data(n, seed):
    rng = np.random.default_rng(seed)
    f = _features(n, seed)
    t = (np.sin(3 * f[:, 0]) + 0.5 * f[:, 3] ** 2 - 2 * f[:, 0] * f[:, 1]).astype(np.float32)
    w = rng.uniform(0.2, 3.0, n).astype(np.float32)
    return f, t, w


@pytest.mark.parametrize("n", [1, 64, 65, 1000, 20_000])
def test_gradient_matches_oracle(ctx, torch_cuda, n):
    torch = torch_cuda
    _say(f"mlp grad n={n}")
    p = _params(4)
    mc.mc_mlp_set(ctx, p.flat())
    f, t, w = _data(n, 10 + n)
    g, loss = mc.mc_mlp_grad(ctx, n, _dev(torch, f), _dev(torch, t), _dev(torch, w))
    f64, t64, w64 = f.astype(np.float64), t.astype(np.float64), w.astype(np.float64)
    y, cache = mlp.forward(p, f64)
    ref = mlp.backward(p, cache, y, t64, w64).flat()
    assert abs(loss - mlp.loss(y, t64, w64)) <= 1e-5 * mlp.loss(y, t64, w64)
    for name, (a, b) in BLOCKS.items():
        scale = np.max(np.abs(ref[a:b]))
        if scale == 0.0:
            continue
        e = np.abs(g[a:b] - ref[a:b]) / scale
        assert np.max(e) <= 2e-3, (name, np.max(e))
        assert np.mean(e <= 2e-4) >= 0.99, (name, np.sort(e)[-10:])


def test_gradient_is_reproducible(ctx, torch_cuda):
    torch = torch_cuda
    mc.mc_mlp_set(ctx, _params(5).flat())
    f, t, w = _data(30_000, 6)
    X, T, W = _dev(torch, f), _dev(torch, t), _dev(torch, w)
    g1, l1 = mc.mc_mlp_grad(ctx, 30_000, X, T, W)
    g2, l2 = mc.mc_mlp_grad(ctx, 30_000, X, T, W)
    assert np.array_equal(g1, g2) and l1 == l2


def test_training_steps_match_oracle(ctx, torch_cuda):
    torch = torch_cuda
    _say("mlp train 10 steps")
    p = _params(6)
    n, steps, lr = 3000, 10, 1e-3
    f, t, w = _data(n, 7)
    mc.mc_mlp_set(ctx, p.flat())
    curve = mc.mc_mlp_train(ctx, n, _dev(torch, f), _dev(torch, t), _dev(torch, w), steps, lr)
    q, ref_curve = mlp.train(p, f.astype(np.float64), t.astype(np.float64), w.astype(np.float64), steps, lr)
    np.testing.assert_allclose(curve, ref_curve, rtol=1e-4)
    d = np.abs(mc.mc_mlp_get(ctx).astype(np.float64) - q.flat())
    assert np.max(d) <= 2 * lr * steps
    assert np.mean(d <= 1e-5) >= 0.99, np.sort(d)[-10:]


def test_training_fits_a_linear_log_importance(ctx, torch_cuda):
    """The pure-absorber shape (ln I linear in depth) is learned to a small
    residual, as by the oracle."""
    torch = torch_cuda
    _say("mlp train 600 steps")
    rng = np.random.default_rng(10)
    n = 4000
    xs = rng.uniform(0, 1, n)
    f = np.stack([xs, rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), rng.uniform(0, 1, n)], 1).astype(np.float32)
    t = (6.0 * xs - 3.0).astype(np.float32)
    w = np.ones(n, np.float32)
    mc.mc_mlp_set(ctx, mlp.init_params(11).flat())
    X = _dev(torch, f)
    curve = mc.mc_mlp_train(ctx, n, X, _dev(torch, t), _dev(torch, w), 600, 1e-2)
    assert curve[-1] < 0.01 * curve[0]
    Y = torch.empty(n, dtype=torch.float32, device="cuda")
    mc.mc_mlp_forward(ctx, n, X, Y)
    torch.cuda.synchronize()
    assert np.sqrt(np.mean((Y.cpu().numpy() - t) ** 2)) < 0.15
