"""FP64 oracle of the importance network -- TEST INFRASTRUCTURE.

The learned importance map is an addition to the paper's method, not part
of the paper: a 4 -> 64 -> 64 -> 1 multilayer perceptron with SiLU hidden
activations that predicts ln I(x, y, z, ln E).  Its kernels on the GPU keep
the weight matrices in BF16, feed BF16 operands to the matrix cores and
accumulate in FP32.  This oracle computes the same network in float64 with
BF16 rounding applied at exactly the kernel's rounding points:

  * the inputs and the three weight matrices W1, W2, w3 are rounded to BF16
    (biases stay FP32 / FP64);
  * the first hidden activation h1 is rounded to BF16 before the 64x64
    product;
  * in the backward pass the gradient dz2 is rounded to BF16 before the two
    products it feeds (dW2 = h1^T dz2 and dh1 = dz2 W2^T);
  * gradients pass through the rounding unchanged (straight-through).

Loss: weighted mean squared error on ln I, sum_i w_i (y_i - t_i)^2 / sum_i w_i.
Optimizer: Adam (Kingma & Ba, 2015) with beta1 0.9, beta2 0.999, eps 1e-8.
``rounding=False`` gives the plain FP64 network (for finite differences).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

N_IN, N_HID = 4, 64


def bf16_round(a) -> np.ndarray:
    """Round float64/float32 values to the nearest BF16 (ties to even), as
    float64.  (FP32 first, then the 16 low bits rounded away.)"""
    f = np.ascontiguousarray(np.asarray(a, np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    if np.any(nan):
        out[nan] = np.nan
    return out.reshape(np.shape(a))


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


@dataclass
class Params:
    W1: np.ndarray  # [4, 64]
    b1: np.ndarray  # [64]
    W2: np.ndarray  # [64, 64]
    b2: np.ndarray  # [64]
    w3: np.ndarray  # [64]
    b3: float

    def copy(self):
        return Params(self.W1.copy(), self.b1.copy(), self.W2.copy(), self.b2.copy(), self.w3.copy(), float(self.b3))

    def flat(self) -> np.ndarray:
        return np.concatenate([self.W1.ravel(), self.b1, self.W2.ravel(), self.b2, self.w3, [self.b3]])

    @staticmethod
    def from_flat(v) -> "Params":
        v = np.asarray(v, np.float64)
        o = 0
        W1 = v[o:o + 256].reshape(4, 64); o += 256
        b1 = v[o:o + 64]; o += 64
        W2 = v[o:o + 4096].reshape(64, 64); o += 4096
        b2 = v[o:o + 64]; o += 64
        w3 = v[o:o + 64]; o += 64
        return Params(W1.copy(), b1.copy(), W2.copy(), b2.copy(), w3.copy(), float(v[o]))


N_PARAMS = 256 + 64 + 4096 + 64 + 64 + 1


def init_params(seed: int = 0) -> Params:
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights, zero biases."""
    rng = np.random.default_rng(seed)
    W1 = rng.uniform(-0.5, 0.5, (4, 64))
    W2 = rng.uniform(-0.125, 0.125, (64, 64))
    w3 = rng.uniform(-0.125, 0.125, 64)
    return Params(W1, np.zeros(64), W2, np.zeros(64), w3, 0.0)


def forward(p: Params, x: np.ndarray, rounding: bool = True):
    """Returns y [n] and the cache for backward."""
    R = bf16_round if rounding else (lambda a: np.asarray(a, np.float64))
    xr = R(x)
    W1, W2, w3 = R(p.W1), R(p.W2), R(p.w3)
    z1 = xr @ W1 + p.b1
    h1 = R(silu(z1))
    z2 = h1 @ W2 + p.b2
    h2 = silu(z2)
    y = h2 @ w3 + p.b3
    return y, (xr, z1, h1, z2, h2, W1, W2, w3, R)


def loss(y, t, w):
    return float(np.sum(w * (y - t) ** 2) / np.sum(w))


def backward(p: Params, cache, y, t, w) -> Params:
    """Gradient of the weighted MSE with respect to every parameter."""
    xr, z1, h1, z2, h2, W1, W2, w3, R = cache
    dy = 2.0 * w * (y - t) / np.sum(w)
    dw3 = h2.T @ dy
    db3 = float(np.sum(dy))
    dz2 = np.outer(dy, w3) * silu_grad(z2)
    dz2r = R(dz2)
    dW2 = h1.T @ dz2r
    db2 = dz2.sum(axis=0)
    dh1 = dz2r @ W2.T
    dz1 = dh1 * silu_grad(z1)
    dW1 = xr.T @ dz1
    db1 = dz1.sum(axis=0)
    return Params(dW1, db1, dW2, db2, dw3, db3)


@dataclass
class Adam:
    lr: float = 1e-3
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    t: int = 0
    m: np.ndarray | None = None
    v: np.ndarray | None = None

    def step(self, p: Params, g: Params) -> Params:
        th, gr = p.flat(), g.flat()
        if self.m is None:
            self.m = np.zeros_like(th)
            self.v = np.zeros_like(th)
        self.t += 1
        self.m = self.beta1 * self.m + (1 - self.beta1) * gr
        self.v = self.beta2 * self.v + (1 - self.beta2) * gr * gr
        mh = self.m / (1 - self.beta1 ** self.t)
        vh = self.v / (1 - self.beta2 ** self.t)
        return Params.from_flat(th - self.lr * mh / (np.sqrt(vh) + self.eps))


def train(p: Params, x, t, w, steps: int, lr: float = 1e-3, rounding: bool = True):
    """Full-batch Adam; returns (params, loss curve before each step)."""
    opt = Adam(lr=lr)
    curve = []
    for _ in range(steps):
        y, cache = forward(p, x, rounding)
        curve.append(loss(y, t, w))
        p = opt.step(p, backward(p, cache, y, t, w))
    return p, np.array(curve)


# feature normalisation of the importance inputs
def features(x, y, z, E, length: float, emin: float = 1e-5, emax: float = 2e7) -> np.ndarray:
    """(x/L, clip(y/L), clip(z/L), (ln E - ln Emin)/ln(Emax/Emin)); y and z are
    clipped to [-1, 1] (the slab is infinite in them)."""
    return np.stack([np.asarray(x, np.float64) / length,
                     np.clip(np.asarray(y, np.float64) / length, -1.0, 1.0),
                     np.clip(np.asarray(z, np.float64) / length, -1.0, 1.0),
                     (np.log(np.asarray(E, np.float64)) - np.log(emin)) / np.log(emax / emin)], axis=-1)
