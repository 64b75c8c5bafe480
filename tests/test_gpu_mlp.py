"""MLP policy trainer on the matrix cores against the oracle (oracle/mlp.py,
the same bf16 roundings, in float64): forward values, one batch's gradient, and
a short training run; the trained weights drive the solver's decision path
bit-exactly.

The matrix cores sum exact bf16 x bf16 products in fp32 in their own order, so
the forward values and gradients are compared element by element against
bounds propagated through the oracle's computation (`bounds` below): a sum of
K products differs by at most gamma_K(fp32) sum |a b| plus the products'
operand perturbations; every bf16 rounding point may land one unit apart
(2^-7 |v|) on top of the perturbation it receives; GELU' <= 1.13 and
|GELU''| <= 0.8 carry perturbations through the activations, and the fp32
GELU and GELU' of the device add 2^-22 |z| (the cancellation in 1 + erf)."""
import numpy as np
import pytest

import oracle as O
from oracle import mlp as L

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    import torch

    import paper_2504_14268_amd as M

    assert torch.cuda.is_available()
    return M


def params(seed):
    p = L.init_params(seed)
    rng = np.random.default_rng(seed + 100)
    for k in ("b1", "b2", "b3"):
        p[k] = (rng.standard_normal(p[k].shape) * 0.1).astype(np.float32).astype(np.float64)
    return p


def data(seed, n):
    rng = np.random.default_rng(seed)
    feat = (rng.standard_normal((n, 16)) * 2).astype(np.float32)
    nxt = (feat + 0.3 * rng.standard_normal((n, 16))).astype(np.float32)
    act = rng.integers(0, 64, n).astype(np.int32)
    rew = (np.tanh(feat[:, 0]) - 0.05 * (act % 16)).astype(np.float32)
    done = (rng.random(n) < 0.1).astype(np.uint8)
    return dict(feat=feat, next=nxt, act=act, rew=rew, done=done)


def dev(M, d):
    import torch

    return {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in d.items()}


U32 = 2.0 ** -24
UNIT = 2.0 ** -7          # one bf16 unit, relative to the value (upper bound)
TINY = 2.0 ** -126


def gam(k):
    return k * U32 / (1 - k * U32)


def bounds(p, feat, act=None, target=None):
    """Oracle values and element-wise bounds of |GPU - oracle| for the forward
    pass (and, with act and target, the loss gradient), propagated through the
    oracle's bf16 forward and backward."""
    B = feat.shape[0]
    r = L.bf16
    x = r(feat.astype(np.float64))
    W1, W2, W3 = r(p["W1"]), r(p["W2"]), r(p["W3"])
    z1 = x @ W1.T + p["b1"]
    e_z1 = gam(17) * (np.abs(x) @ np.abs(W1).T + np.abs(p["b1"]))
    h1 = r(L.gelu(z1))
    e_h1 = UNIT * np.abs(h1) + 1.13 * e_z1 + 1e-6 * np.abs(L.gelu(z1)) + 2.0 ** -22 * np.abs(z1) + TINY
    z2 = h1 @ W2.T + p["b2"]
    e_z2 = gam(129) * (np.abs(h1) @ np.abs(W2).T + np.abs(p["b2"])) + e_h1 @ np.abs(W2).T
    h2 = r(L.gelu(z2))
    e_h2 = UNIT * np.abs(h2) + 1.13 * e_z2 + 1e-6 * np.abs(L.gelu(z2)) + 2.0 ** -22 * np.abs(z2) + TINY
    y = h2 @ W3.T + p["b3"]
    e_y = gam(129) * (np.abs(h2) @ np.abs(W3).T + np.abs(p["b3"])) + e_h2 @ np.abs(W3).T
    out = dict(y=y, e_y=e_y)
    if act is None:
        return out
    rows = np.arange(B)
    diff = y[rows, act] - target
    e_diff = e_y[rows, act]
    out["loss"] = 0.5 * np.mean(diff ** 2)
    out["e_loss"] = np.mean(np.abs(diff) * e_diff + 0.5 * e_diff ** 2) + gam(B) * out["loss"]
    dY = np.zeros_like(y)
    e_dY = np.zeros_like(y)
    dY[rows, act] = diff / B
    e_dY[rows, act] = e_diff / B
    dYr = r(dY)
    e_dYr = e_dY + UNIT * np.abs(dY) + TINY * (dY != 0)
    g, e = {}, {}
    g["W3"] = dYr.T @ h2
    e["W3"] = gam(B) * (np.abs(dYr).T @ np.abs(h2)) + e_dYr.T @ (np.abs(h2) + e_h2) + np.abs(dYr).T @ e_h2
    g["b3"] = dY.sum(axis=0)
    e["b3"] = e_dY.sum(axis=0) + gam(B) * np.abs(dY).sum(axis=0)
    gp2 = L.gelu_grad(z2)
    t2 = dYr @ W3
    e_t2 = e_dYr @ np.abs(W3) + gam(65) * (np.abs(dYr) @ np.abs(W3))
    dZ2 = t2 * gp2
    e_dZ2 = e_t2 * (np.abs(gp2) + 0.8 * e_z2) + np.abs(t2) * (0.8 * e_z2 + 1e-6 + 2.0 ** -22 * np.abs(z2)) + U32 * np.abs(dZ2)
    dZ2r = r(dZ2)
    e_dZ2r = e_dZ2 + UNIT * np.abs(dZ2) + TINY
    g["W2"] = dZ2r.T @ h1
    e["W2"] = gam(B) * (np.abs(dZ2r).T @ np.abs(h1)) + e_dZ2r.T @ (np.abs(h1) + e_h1) + np.abs(dZ2r).T @ e_h1
    g["b2"] = dZ2.sum(axis=0)
    e["b2"] = e_dZ2.sum(axis=0) + gam(B) * np.abs(dZ2).sum(axis=0)
    gp1 = L.gelu_grad(z1)
    t1 = dZ2r @ W2
    e_t1 = e_dZ2r @ np.abs(W2) + gam(129) * (np.abs(dZ2r) @ np.abs(W2))
    dZ1 = t1 * gp1
    e_dZ1 = e_t1 * (np.abs(gp1) + 0.8 * e_z1) + np.abs(t1) * (0.8 * e_z1 + 1e-6 + 2.0 ** -22 * np.abs(z1)) + U32 * np.abs(dZ1)
    dZ1r = r(dZ1)
    e_dZ1r = e_dZ1 + UNIT * np.abs(dZ1) + TINY
    g["W1"] = dZ1r.T @ x
    e["W1"] = gam(B) * (np.abs(dZ1r).T @ np.abs(x)) + e_dZ1r.T @ np.abs(x)
    g["b1"] = dZ1.sum(axis=0)
    e["b1"] = e_dZ1.sum(axis=0) + gam(B) * np.abs(dZ1).sum(axis=0)
    out["g"], out["e"] = g, e
    return out


def test_bounds_reduce_to_oracle():
    """The bounded quantities are the oracle's own: same forward, same gradient."""
    p = params(3)
    d = data(4, 128)
    tgt = np.random.default_rng(5).standard_normal(128)
    bo = bounds(p, d["feat"], d["act"], tgt)
    y, _ = L.forward(p, d["feat"].astype(np.float64))
    lo, go = L.loss_and_grads(p, d["feat"].astype(np.float64), d["act"], tgt)
    assert np.array_equal(bo["y"], y) and bo["loss"] == lo
    for k in go:
        assert np.allclose(bo["g"][k], go[k], rtol=1e-12, atol=1e-300), k


def test_forward_matches_oracle(M):
    p = params(1)
    net = M.Mlp(p)
    d = data(2, 300)               # not a multiple of the 64-sample tile
    g = net.forward(dev(M, d)["feat"]).cpu().numpy().astype(np.float64)
    bo = bounds(p, d["feat"])
    err = np.abs(g - bo["y"])
    assert np.all(err <= bo["e_y"]), float(np.max(err / bo["e_y"]))
    # most values agree to well inside one bf16 unit of the output
    assert np.median(err / np.maximum(np.abs(bo["y"]), 1e-30)) <= 2.0 ** -9


def test_grad_matches_oracle(M):
    p = params(3)
    net = M.Mlp(p)
    d = data(4, 256)
    tgt = np.random.default_rng(5).standard_normal(256).astype(np.float32)
    dd = dev(M, dict(feat=d["feat"], act=d["act"], tgt=tgt))
    g, loss = net.grad(dd["feat"], dd["act"], dd["tgt"])
    bo = bounds(p, d["feat"], d["act"], tgt.astype(np.float64))
    assert abs(loss - bo["loss"]) <= bo["e_loss"] + U32 * abs(bo["loss"])
    for k in bo["g"]:
        err = np.abs(g[k].astype(np.float64) - bo["g"][k])
        assert np.all(err <= bo["e"][k] + U32 * np.abs(bo["g"][k])), (k, float(np.max(err / (bo["e"][k] + 1e-300))))


def test_training_matches_oracle(M):
    p = params(6)
    d = data(7, 1024)
    net = M.Mlp(p)
    losses = net.train(dev(M, d), batch=256, epochs=3, lr=1e-3, gamma=0.9)
    po = {k: v.copy() for k, v in p.items()}
    od = {k: v.astype(np.float64) if v.dtype != np.int32 else v for k, v in d.items()}
    lo = L.train(po, od, batch=256, epochs=3, gamma=0.9, lr=1e-3)
    assert np.allclose(losses, lo, rtol=3e-2)
    assert losses[-1] < losses[0]
    g = net.params()
    steps = 3 * (1024 // 256)
    for k in p:
        moved = np.linalg.norm(po[k] - p[k])
        assert np.linalg.norm(g[k] - po[k]) <= 0.1 * moved + 1e-7, k
        # element by element: an Adam step moves a parameter by at most about
        # lr (1 - b1) / sqrt(1 - b2) < 3.2 lr, so the two runs, from the same
        # start, stay within 2 x 3.2 lr per step of each other
        assert np.all(np.abs(g[k] - po[k]) <= 2 * 3.2 * 1e-3 * steps), k


def test_trained_net_drives_decisions(M):
    p = params(8)
    net = M.Mlp(p)
    net.train(dev(M, data(9, 512)), batch=128, epochs=2)
    P = M.Policy(kind=M.POLICY_MLP)
    net.to_policy(P)
    w = net.params()
    wb = {k: (O.rd(v.astype(np.float64).ravel(), O.BF16).reshape(v.shape).astype(np.float32) if k.startswith("W") else v)
          for k, v in w.items()}
    op = O.OraclePolicy(kind=O.POL_MLP, mlp=wb)
    rng = np.random.default_rng(10)
    feat = (rng.standard_normal((40, 16)) * 2).astype(np.float32)
    k = np.arange(40, dtype=np.int64)
    rho = np.full(40, 1e-3)
    stag = np.zeros(40, np.int32)
    _, acts = P.decide(k, rho, stag, feat)
    for i in range(40):
        assert acts[i] == int(np.argmax(op.mlp_logits(feat[i])))
