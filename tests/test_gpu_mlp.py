"""MLP policy trainer on the matrix cores against the oracle (oracle/mlp.py,
the same roundings in float64): forward values, one batch's gradient, and a
short training run; the trained weights drive the solver's decision path
bit-exactly.  Matrix-core accumulation order differs from the oracle's, and a
bf16 activation can move by one unit, so the bounds are relative to the
values' scale (a few bf16 units)."""
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


def test_forward_matches_oracle(M):
    p = params(1)
    net = M.Mlp(p)
    d = data(2, 300)               # not a multiple of the 64-sample tile
    g = net.forward(dev(M, d)["feat"]).cpu().numpy().astype(np.float64)
    o, _ = L.forward(p, d["feat"].astype(np.float64))
    scale = np.abs(o).max()
    err = np.abs(g - o)
    assert err.max() <= 2e-2 * scale
    assert np.median(err) <= 1e-4 * scale


def test_grad_matches_oracle(M):
    p = params(3)
    net = M.Mlp(p)
    d = data(4, 256)
    tgt = np.random.default_rng(5).standard_normal(256).astype(np.float32)
    dd = dev(M, dict(feat=d["feat"], act=d["act"], tgt=tgt))
    g, loss = net.grad(dd["feat"], dd["act"], dd["tgt"])
    lo, go = L.loss_and_grads(p, d["feat"].astype(np.float64), d["act"], tgt.astype(np.float64))
    assert abs(loss - lo) <= 1e-3 * abs(lo)
    for k in go:
        den = np.linalg.norm(go[k])
        assert np.linalg.norm(g[k] - go[k]) <= 3e-2 * den + 1e-9, k


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
    for k in p:
        moved = np.linalg.norm(po[k] - p[k])
        assert np.linalg.norm(g[k] - po[k]) <= 0.1 * moved + 1e-7, k


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
