"""Oracle of the MLP precision policy's training step.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may use this module; the GPU library does not.

Plain numpy in float64.  The network is the policy network of the decision
path (16 features -> 128 -> 128 -> 64 action values, GELU by Abramowitz &
Stegun 7.1.28), trained by fitted Q-iteration, the function-approximation form
of the Q-learning update of section 4.1:

    target  y_t = r_t + gamma (1 - done_t) max_a' Q_frozen(s_{t+1}, a')
    loss    L = mean over the batch of 1/2 (Q(s_t, a_t) - y_t)^2

(only the taken action's value receives a gradient), minimised by Adam
(Kingma & Ba 2015) on float master weights.

With `emulate=True` the forward and backward passes round to bfloat16 exactly
where the matrix-core kernels take bfloat16 operands: the input features, the
weights, both hidden activations, and the gradient operands dY, dZ2, dZ1 of
the backward products.  Bias gradients and the GELU derivative use the
unrounded values.  Every rounding is passed through (its derivative is 1).
With `emulate=False` everything is float64, which is what the finite-difference
checks use.
"""
from __future__ import annotations

import numpy as np

from . import BF16, rd

IN, HID, NACT = 16, 128, 64
A_S = (0.0705230784, 0.0422820123, 0.0092705272, 0.0001520143, 0.0002765672, 0.0000430638)
SQRT_HALF = 0.70710678118654752440


def bf16(x):
    """Round to bfloat16 (round to nearest even, directly from float64)."""
    x = np.asarray(x, dtype=np.float64)
    return rd(x.ravel(), BF16).reshape(x.shape)


def _erf_parts(t):
    """d(t) = 1 + a1 t + ... + a6 t^6 and d'(t), t >= 0 (A&S 7.1.28: erf = 1 - d^-16)."""
    a1, a2, a3, a4, a5, a6 = A_S
    d = 1.0 + t * (a1 + t * (a2 + t * (a3 + t * (a4 + t * (a5 + t * a6)))))
    dd = a1 + t * (2 * a2 + t * (3 * a3 + t * (4 * a4 + t * (5 * a5 + t * 6 * a6))))
    return d, dd


def gelu(x):
    """x/2 (1 + erf(x / sqrt 2)), erf by A&S 7.1.28."""
    x = np.asarray(x, dtype=np.float64)
    z = x * SQRT_HALF
    d, _ = _erf_parts(np.abs(z))
    erf = np.sign(z) * (1.0 - d ** -16)
    return 0.5 * x * (1.0 + erf)


def gelu_grad(x):
    """Exact derivative of `gelu` as defined above (A&S erf included)."""
    x = np.asarray(x, dtype=np.float64)
    z = x * SQRT_HALF
    t = np.abs(z)
    d, dd = _erf_parts(t)
    erf = np.sign(z) * (1.0 - d ** -16)
    derf = 16.0 * dd * d ** -17          # d erf / dz, an even function of z
    return 0.5 * (1.0 + erf) + 0.5 * x * derf * SQRT_HALF


def init_params(seed: int) -> dict:
    """He-style initial weights (float32 values), zero biases."""
    rng = np.random.default_rng(seed)
    f = lambda a: a.astype(np.float32).astype(np.float64)
    return dict(W1=f(rng.standard_normal((HID, IN)) * np.sqrt(2.0 / IN)), b1=np.zeros(HID),
                W2=f(rng.standard_normal((HID, HID)) * np.sqrt(2.0 / HID)), b2=np.zeros(HID),
                W3=f(rng.standard_normal((NACT, HID)) * np.sqrt(1.0 / HID)), b3=np.zeros(NACT))


def forward(p: dict, feat, emulate: bool = True):
    """Action values Y[B, 64] of features feat[B, 16]; returns (Y, cache)."""
    r = bf16 if emulate else (lambda v: np.asarray(v, dtype=np.float64))
    x = r(feat)
    W1, W2, W3 = r(p["W1"]), r(p["W2"]), r(p["W3"])
    z1 = x @ W1.T + p["b1"]
    h1 = r(gelu(z1))
    z2 = h1 @ W2.T + p["b2"]
    h2 = r(gelu(z2))
    y = h2 @ W3.T + p["b3"]
    return y, dict(x=x, z1=z1, h1=h1, z2=z2, h2=h2, W1=W1, W2=W2, W3=W3)


def targets(p_frozen: dict, next_feat, rew, done, gamma: float, emulate: bool = True):
    """y_t = r_t + gamma (1 - done_t) max_a Q_frozen(s_{t+1}, a)."""
    y, _ = forward(p_frozen, next_feat, emulate)
    return np.asarray(rew, dtype=np.float64) + gamma * (1.0 - np.asarray(done, dtype=np.float64)) * y.max(axis=1)


def loss_and_grads(p: dict, feat, act, target, emulate: bool = True):
    """Mean 1/2 (Q(s, a) - y)^2 over the batch and its gradient for every parameter."""
    r = bf16 if emulate else (lambda v: np.asarray(v, dtype=np.float64))
    feat = np.asarray(feat, dtype=np.float64)
    act = np.asarray(act, dtype=np.int64)
    B = feat.shape[0]
    y, c = forward(p, feat, emulate)
    q = y[np.arange(B), act]
    diff = q - np.asarray(target, dtype=np.float64)
    loss = 0.5 * np.mean(diff * diff)
    dY = np.zeros_like(y)
    dY[np.arange(B), act] = diff / B
    dYr = r(dY)
    g = {}
    g["W3"] = dYr.T @ c["h2"]
    g["b3"] = dY.sum(axis=0)
    dZ2 = (dYr @ c["W3"]) * gelu_grad(c["z2"])
    dZ2r = r(dZ2)
    g["W2"] = dZ2r.T @ c["h1"]
    g["b2"] = dZ2.sum(axis=0)
    dZ1 = (dZ2r @ c["W2"]) * gelu_grad(c["z1"])
    dZ1r = r(dZ1)
    g["W1"] = dZ1r.T @ c["x"]
    g["b1"] = dZ1.sum(axis=0)
    return loss, g


class Adam:
    """Adam on a dict of float arrays (lr 1e-3, betas 0.9 / 0.999, eps 1e-8)."""

    def __init__(self, p: dict, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.m = {k: np.zeros_like(v) for k, v in p.items()}
        self.v = {k: np.zeros_like(v) for k, v in p.items()}
        self.t = 0

    def step(self, p: dict, g: dict):
        self.t += 1
        c1 = 1.0 - self.b1 ** self.t
        c2 = 1.0 - self.b2 ** self.t
        for k in p:
            self.m[k] = self.b1 * self.m[k] + (1.0 - self.b1) * g[k]
            self.v[k] = self.b2 * self.v[k] + (1.0 - self.b2) * g[k] * g[k]
            p[k] = p[k] - self.lr * (self.m[k] / c1) / (np.sqrt(self.v[k] / c2) + self.eps)


def train(p: dict, data: dict, batch: int, epochs: int, gamma: float = 0.9, emulate: bool = True, **adam):
    """Fitted Q-iteration: per epoch, targets from the weights frozen at its
    start, then Adam steps over consecutive batches of the data in order."""
    opt = Adam(p, **adam)
    n = len(data["act"])
    losses = []
    for _ in range(epochs):
        frozen = {k: v.copy() for k, v in p.items()}
        y = targets(frozen, data["next"], data["rew"], data["done"], gamma, emulate)
        tot = 0.0
        for s in range(0, n - batch + 1, batch):
            sl = slice(s, s + batch)
            loss, g = loss_and_grads(p, data["feat"][sl], data["act"][sl], y[sl], emulate)
            opt.step(p, g)
            tot += loss
        losses.append(tot / max(1, n // batch))
    return losses
