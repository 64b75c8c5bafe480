"""Pins of the MLP training oracle (oracle/mlp.py): its GELU against the C
oracle's and against erf, its analytic gradients against central finite
differences in float64, Adam's first step against its closed form, the targets
by hand, and the emulated forward pass against the C decision path."""
import math

import numpy as np
import pytest

import oracle as O
from oracle import mlp as L


def test_gelu_matches_c_oracle_and_erf():
    xs = np.linspace(-7, 7, 2001)
    g = L.gelu(xs)
    c = np.array([O.gelu(float(np.float32(x))) for x in xs])
    assert np.max(np.abs(g - c)) <= 1e-6 * np.maximum(1.0, np.abs(xs)).max()
    exact = np.array([0.5 * x * (1 + math.erf(x / math.sqrt(2))) for x in xs])
    assert np.max(np.abs(g - exact) / np.maximum(1.0, np.abs(xs))) < 2e-7   # A&S 7.1.28: |err| <= 3e-7


def test_gelu_grad_finite_differences():
    xs = np.concatenate([np.linspace(-6, 6, 601), [1e-3, -1e-3]])
    h = 1e-6
    fd = (L.gelu(xs + h) - L.gelu(xs - h)) / (2 * h)
    assert np.max(np.abs(L.gelu_grad(xs) - fd)) < 1e-8
    assert abs(L.gelu_grad(0.0) - 0.5) < 1e-15


def _small_problem(seed=0, B=8):
    rng = np.random.default_rng(seed)
    p = L.init_params(seed)
    for k in ("b1", "b2", "b3"):
        p[k] = rng.standard_normal(p[k].shape) * 0.1
    feat = rng.standard_normal((B, 16)) * 2
    act = rng.integers(0, 64, B)
    tgt = rng.standard_normal(B)
    return p, feat, act, tgt


def test_backward_finite_differences():
    p, feat, act, tgt = _small_problem()
    loss, g = L.loss_and_grads(p, feat, act, tgt, emulate=False)
    rng = np.random.default_rng(9)
    h = 1e-6
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        for _ in range(12):
            idx = tuple(rng.integers(0, s) for s in p[k].shape)
            if k == "W3" or k == "b3":   # only the taken actions' rows carry gradient
                idx = (int(act[rng.integers(0, len(act))]),) + idx[1:]
            old = p[k][idx]
            p[k][idx] = old + h
            lp, _ = L.loss_and_grads(p, feat, act, tgt, emulate=False)
            p[k][idx] = old - h
            lm, _ = L.loss_and_grads(p, feat, act, tgt, emulate=False)
            p[k][idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(g[k][idx] - fd) <= 1e-6 * max(1e-3, abs(fd)), (k, idx, g[k][idx], fd)


def test_untaken_actions_get_no_gradient():
    p, feat, act, tgt = _small_problem(1)
    _, g = L.loss_and_grads(p, feat, act, tgt)
    untaken = np.setdiff1d(np.arange(64), act)
    assert np.all(g["W3"][untaken] == 0) and np.all(g["b3"][untaken] == 0)


def test_adam_first_step_closed_form():
    p, feat, act, tgt = _small_problem(2)
    _, g = L.loss_and_grads(p, feat, act, tgt)
    p0 = {k: v.copy() for k, v in p.items()}
    opt = L.Adam(p, lr=1e-3)
    opt.step(p, g)
    for k in p:
        expect = p0[k] - 1e-3 * g[k] / (np.abs(g[k]) + 1e-8)
        assert np.allclose(p[k], expect, rtol=0, atol=1e-15)


def test_targets_by_hand():
    p = L.init_params(3)
    nxt = np.random.default_rng(4).standard_normal((3, 16))
    y, _ = L.forward(p, nxt)
    t = L.targets(p, nxt, [1.0, 2.0, -0.5], [1, 0, 0], 0.9)
    assert t[0] == 1.0
    assert t[1] == 2.0 + 0.9 * y[1].max() and t[2] == -0.5 + 0.9 * y[2].max()


def test_emulated_forward_matches_decision_path():
    p = L.init_params(5)
    w = {k: (L.bf16(v) if k.startswith("W") else v).astype(np.float32) for k, v in p.items()}
    w["b1"] = (np.random.default_rng(6).standard_normal(128) * 0.1).astype(np.float32)
    pol = O.OraclePolicy(kind=O.POL_MLP, mlp=w)
    q = {k: v.astype(np.float64) for k, v in w.items()}
    rng = np.random.default_rng(7)
    feats = (rng.standard_normal((50, 16)) * 3).astype(np.float32)
    y, _ = L.forward(q, feats.astype(np.float64))
    for i in range(50):
        c = pol.mlp_logits(feats[i]).astype(np.float64)
        scale = np.abs(y[i]).max()
        # identical roundings; only the accumulation (fp32 chains vs float64)
        # differs, which can move a bf16 activation by one unit now and then
        assert np.max(np.abs(c - y[i])) <= 2e-2 * scale, i


def test_training_lowers_the_loss():
    rng = np.random.default_rng(8)
    n = 512
    feat = rng.standard_normal((n, 16))
    act = rng.integers(0, 64, n)
    rew = np.tanh(feat[:, 0] + 0.5 * feat[:, 1]) + 0.1 * (act % 4)
    data = dict(feat=feat, next=feat, act=act, rew=rew, done=np.ones(n))
    p = L.init_params(10)
    losses = L.train(p, data, batch=64, epochs=6, gamma=0.9, lr=3e-3)
    assert losses[-1] < 0.5 * losses[0]
