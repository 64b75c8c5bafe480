"""Tabular Q-learning over several systems through mpcg_train_qlearning
(section 4.1, Algorithm 1): every episode's solve and the final Q-table equal
the oracle's, bit for bit, when the oracle runs the same episodes in the same
order with the same epsilon schedule and episode numbers."""
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


def systems():
    out = []
    A = W.laplacian_2d(24)
    out.append((A, W.rhs(A.n, 41)))
    A = W.random_spd(3000, 42, W.spread_for_kappa(1e4))
    out.append((A, W.rhs(A.n, 43)))
    A = W.banded_spd(2500, 3, 44, W.spread_for_kappa(1e3))
    out.append((A, W.rhs(A.n, 45)))
    return out


def schedule(e, total, es, ee):
    return es + (ee - es) * (e - 1) / (total - 1) if total > 1 else es


@pytest.mark.parametrize("order,cost,first", [(0, "C1", 1), (1, "C2", 4)])
def test_train_matches_oracle(M, order, cost, first):
    import torch

    sysl = systems()
    E, maxit, tol, es, ee, seed = 3, 300, 1e-8, 1.0, 0.1, 901
    P = M.Policy(kind=M.POLICY_QTABLE_TRAIN, cost=cost, seed=seed)
    gs = []
    for A, b in sysl:
        m = M.Matrix(A)
        m.set_options(replace_period=50, fallback=True)
        gs.append((m, torch.from_numpy(b).cuda(), torch.empty(A.n, dtype=torch.float64, device="cuda")))
    total = first - 1 + len(sysl) * E + 2          # a schedule longer than this call
    out = M.train_qlearning(P, gs, episodes=E, maxit=maxit, tol=tol, eps_start=es, eps_end=ee,
                            order=order, first_episode=first, total_episodes=total)
    op = O.OraclePolicy(kind=O.POL_QTRAIN, cost=cost, seed=seed)
    m_ = len(sysl)
    for j in range(m_ * E):
        s = j // E if order == 0 else j % m_
        e = first + j
        eps = schedule(e, total, es, ee)
        op.s.episode, op.s.epsilon = e, eps
        A, b = sysl[s]
        xo, info = O.cg(A, b, tol=tol, maxit=maxit, policy=op, replace_period=50, fallback=True)
        r = out[j]
        assert (r["system"], r["episode"]) == (s, e)
        assert r["epsilon"] == eps
        assert (r["status"], r["iters"], r["n_replace"], r["fallback_at"]) == \
            (info["status"], info["iters"], info["n_replace"], info["fallback_at"]), (j, r, info)
        assert r["cost_sum"] == info["cost_sum"]
        assert r["relres_true"] == info["relres_true"] or (np.isnan(r["relres_true"]) and np.isnan(info["relres_true"]))
        if j == m_ * E - 1:
            assert np.array_equal(gs[s][2].cpu().numpy(), xo)
    assert np.array_equal(P.qtable(), op.q)
    assert np.count_nonzero(op.q) > 0


def test_train_rejects_bad_descriptor(M):
    import torch

    A = W.laplacian_2d(8)
    m = M.Matrix(A)
    b = torch.from_numpy(W.rhs(A.n, 1)).cuda()
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    P = M.Policy(kind=M.POLICY_QTABLE_TRAIN)
    with pytest.raises(M.MPCGError):
        M.train_qlearning(P, [(m, b, x)], episodes=0)
    with pytest.raises(M.MPCGError):
        M.train_qlearning(P, [(m, b, x)], eps_start=1.5)
    with pytest.raises(M.MPCGError):
        M.train_qlearning(M.Policy(kind=M.POLICY_QTABLE), [(m, b, x)])
