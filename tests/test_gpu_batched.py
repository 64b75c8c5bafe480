"""Batched persistent solve (mpcg_solve_batched): every system's result equals
its own mpcg_solve and the oracle's, bit for bit, for several launch
configurations and the autotuner's choice (batch invariance)."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    import torch

    import paper_2504_14268_amd as M

    assert torch.cuda.is_available()
    return M


def batch_systems():
    """Uneven sizes and families: banded and random-pattern SPD, a Laplacian, a
    1x1 system and a ragged tiny one."""
    out = []
    for sd in range(1000, 1008):
        A = W.batch_system(sd, n_lo=100, n_hi=20000)
        out.append((A, W.rhs(A.n, sd + 5000)))
    A = W.laplacian_2d(37)
    out.append((A, W.rhs(A.n, 7)))
    out.append((W.CSR(1, np.array([0, 1], np.int32), np.array([0], np.int32), np.array([3.0])), np.array([1.5])))
    A = W.random_spd(37, 9, 1.0)
    out.append((A, W.rhs(A.n, 10)))
    A = W.random_spd(5000, 11, W.spread_for_kappa(1e5))
    out.append((A, W.rhs(A.n, 12)))
    return out


def policies(M, n):
    from test_oracle_policy import mlp_weights

    rng = np.random.default_rng(5)
    q = rng.standard_normal((100, 64))
    w = mlp_weights(3)
    gp, op = [], []
    for i in range(n):
        kind = i % 4
        if kind == 0:
            a = M.action(M.BF16, M.FP32, M.FP32)
            gp.append(M.Policy(kind=M.POLICY_FIXED, fixed_action=a))
            op.append(O.OraclePolicy(fixed_action=a))
        elif kind == 1:
            gp.append(M.Policy(kind=M.POLICY_FIXED, fixed_action=63))
            op.append(O.OraclePolicy(fixed_action=63))
        elif kind == 2:
            P = M.Policy(kind=M.POLICY_QTABLE)
            P.set_qtable(q)
            gp.append(P)
            op.append(O.OraclePolicy(kind=O.POL_QTABLE, q=q))
        else:
            P = M.Policy(kind=M.POLICY_MLP)
            P.set_mlp(w)
            gp.append(P)
            op.append(O.OraclePolicy(kind=O.POL_MLP, mlp=w))
    return gp, op


def run_batch(M, sysl, gp, cfgs, maxit=600):
    import torch

    mats, bs = [], []
    for (A, b), P in zip(sysl, gp):
        m = M.Matrix(A)
        m.set_policy(P)
        m.set_options(replace_period=50, fallback=True)
        mats.append(m)
        bs.append(torch.from_numpy(b).cuda())
    outs = []
    for cfg in cfgs:
        xs = [torch.zeros(A.n, dtype=torch.float64, device="cuda") for A, _ in sysl]
        res, info = M.solve_batched([(m, b, x) for m, b, x in zip(mats, bs, xs)], tol=1e-8, maxit=maxit, **cfg)
        hist = [m.history() for m in mats]
        outs.append((res, info, [x.cpu().numpy() for x in xs], hist))
    # single solves of the same systems
    single = []
    for m, b, (A, _) in zip(mats, bs, sysl):
        x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        r = m.solve(b, x, tol=1e-8, maxit=maxit)
        single.append((r, x.cpu().numpy(), m.history()))
    return outs, single


def same(r1, x1, h1, r2, x2, h2):
    for key in ("status", "iters", "n_replace", "fallback_at", "cost_sum"):
        assert r1[key] == r2[key], (key, r1, r2)
    assert r1["relres_true"] == r2["relres_true"] or (np.isnan(r1["relres_true"]) and np.isnan(r2["relres_true"]))
    k = r1["iters"]
    assert np.array_equal(h1["rho"][:k + 1], h2["rho"][:k + 1], equal_nan=True)
    assert np.array_equal(h1["actions"][:k], h2["actions"][:k])
    assert np.array_equal(h1["flags"][:k], h2["flags"][:k])
    assert np.array_equal(x1, x2)


def test_batched_equals_single_and_oracle(M):
    sysl = batch_systems()
    gp, op = policies(M, len(sysl))
    cfgs = [dict(workgroups=3, spmv_rows=512, split_rows=-1, strategy=1),
            dict(workgroups=64, spmv_rows=2048, order=1, split_rows=-1, strategy=1),
            dict(workgroups=16, spmv_rows=1024, split_rows=3000, strategy=1),
            dict(spmv_rows=512, strategy=2), dict(spmv_rows=2048, strategy=2, order=1), dict()]
    outs, single = run_batch(M, sysl, gp, cfgs)
    for (res, info, xs, hist), cfg in zip(outs, cfgs):
        assert info["workgroups"] > 0 and info["spmv_rows"] in (512, 1024, 2048)
        if cfg.get("strategy"):
            assert info["strategy"] == cfg["strategy"]
        for i in range(len(sysl)):
            same(res[i], xs[i], hist[i], *single[i])
    assert outs[2][1]["n_split"] == sum(1 for A, _ in sysl if A.n > 3000) > 0
    assert outs[5][1]["tuned"] in (1, 2)
    for i, ((A, b), P) in enumerate(zip(sysl, op)):
        xo, info = O.cg(A, b, tol=1e-8, maxit=600, policy=P, replace_period=50, fallback=True)
        r, x, h = single[i]
        assert (r["status"], r["iters"]) == (info["status"], info["iters"]), i
        assert np.array_equal(x, xo), i


def test_batched_fallback_and_budget(M):
    A = W.random_spd(2000, 31, spread=3.0)
    b = W.rhs(A.n, 32) * 1e6
    sysl = [(A, b), (W.laplacian_2d(30), W.rhs(900, 3))]
    gp = [M.Policy(kind=M.POLICY_FIXED, fixed_action=0), M.Policy(kind=M.POLICY_FIXED, fixed_action=21)]
    outs, single = run_batch(M, sysl, gp, [dict(workgroups=2, spmv_rows=1024, split_rows=-1, strategy=1),
                                           dict(spmv_rows=1024, strategy=2)], maxit=40)
    for res, info, xs, hist in outs:
        for i in range(2):
            same(res[i], xs[i], hist[i], *single[i])


def test_batched_rejects(M):
    import torch

    A = W.laplacian_2d(8)
    m = M.Matrix(A)
    b = torch.from_numpy(W.rhs(A.n, 1)).cuda()
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    with pytest.raises(M.MPCGError):
        M.solve_batched([(m, b, x), (m, b, x)])
    m.set_policy(M.Policy(kind=M.POLICY_QTABLE_TRAIN))
    with pytest.raises(M.MPCGError):
        M.solve_batched([(m, b, x)])
    m.set_policy(None)
    with pytest.raises(M.MPCGError):
        M.solve_batched([(m, b, x)], spmv_rows=300)
    res, info = M.solve_batched([])
    assert res == []
