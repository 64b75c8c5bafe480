"""GPU parity of the decision period (the policy acts every D iterations and
its action holds in between; one Q update and one rollout per decision):
Q-learning episodes (the Q-table and rollouts after every episode), a greedy
table with a period that is not a multiple of the replacement period, and the
network policy -- bit for bit against the oracle."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def M():
    import paper_2504_14268_amd as M

    M.lib()
    assert torch.cuda.is_available()
    return M


def run(M, m, A, b, P, op, maxit, fallback=True, roll=0):
    m.set_policy(P)
    m.set_options(replace_period=50, fallback=fallback)
    xd = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    res = m.solve(torch.from_numpy(b).cuda(), xd, tol=1e-8, maxit=maxit)
    h = m.history()
    xo, info = O.cg(A, b, tol=1e-8, maxit=maxit, policy=op, replace_period=50, fallback=fallback, roll_cap=roll)
    k = info["iters"]
    assert (res["status"], res["iters"], res["fallback_at"]) == (info["status"], k, info["fallback_at"])
    assert np.array_equal(h["rho"][:k + 1], info["rho"][:k + 1])
    assert np.array_equal(h["actions"][:k], info["actions"][:k])
    assert np.array_equal(h["flags"][:k], info["flags"][:k])
    assert res["cost_sum"] == info["cost_sum"] and np.array_equal(xd.cpu().numpy(), xo)
    return info


@pytest.mark.parametrize("D", [50, 7])
def test_qlearning_with_decision_period(M, D):
    A = W.random_spd(15000, 41, W.spread_for_kappa(1e5))
    b = W.rhs(A.n, 42)
    P = M.Policy(kind=M.POLICY_QTABLE_TRAIN, cost="C1", seed=9, decision_period=D)
    P.rollouts_enable(5000)
    op = O.OraclePolicy(kind=O.POL_QTRAIN, cost="C1", seed=9, decision_period=D)
    m = M.Matrix(A)
    rolls = []
    for e in (1, 2, 3):
        eps = 1.0 - 0.45 * (e - 1)
        P.set_episode(e, eps)
        op.s.episode, op.s.epsilon = e, eps
        info = run(M, m, A, b, P, op, 700, roll=5000)
        assert np.array_equal(P.qtable(), op.q)
        rolls.append(info["rollouts"])
    g = P.rollouts()
    for key in ("feat", "next", "act", "rew", "done"):
        assert np.array_equal(g[key], np.concatenate([r[key] for r in rolls]))


def test_greedy_table_with_decision_period(M):
    rng = np.random.default_rng(17)
    q = rng.standard_normal((100, 64))
    A = W.random_spd(20000, 43, W.spread_for_kappa(1e4))
    b = W.rhs(A.n, 44)
    P = M.Policy(kind=M.POLICY_QTABLE, decision_period=7)
    P.set_qtable(q)
    info = run(M, M.Matrix(A), A, b, P, O.OraclePolicy(kind=O.POL_QTABLE, q=q, decision_period=7), 1500)
    acts = info["actions"]
    assert all(acts[i] == acts[i - 1] for i in range(1, len(acts)) if i % 7 and i != info["fallback_at"])


def test_network_policy_with_decision_period(M):
    from test_oracle_policy import mlp_weights

    w = mlp_weights(11)
    A = W.random_spd(12000, 45, W.spread_for_kappa(1e4))
    b = W.rhs(A.n, 46)
    P = M.Policy(kind=M.POLICY_MLP, decision_period=10)
    P.set_mlp(w)
    P.rollouts_enable(2000)
    run(M, M.Matrix(A), A, b, P, O.OraclePolicy(kind=O.POL_MLP, mlp=w, decision_period=10), 800, roll=2000)


@pytest.mark.parametrize("D", [1, 50])
def test_per_op_tables_qlearning_and_greedy(M, D):
    """One Q-table per operation: training episodes (tables and rollouts after
    each), then the greedy policy and its decisions, equal the oracle's."""
    A = W.random_spd(12000, 47, W.spread_for_kappa(1e5))
    b = W.rhs(A.n, 48)
    P = M.Policy(kind=M.POLICY_QTABLE_TRAIN, cost="C2", seed=13, decision_period=D, per_op=1)
    op = O.OraclePolicy(kind=O.POL_QTRAIN, cost="C2", seed=13, decision_period=D, per_op=1)
    m = M.Matrix(A)
    for e in (1, 2, 3):
        eps = 1.0 - 0.4 * (e - 1)
        P.set_episode(e, eps)
        op.s.episode, op.s.epsilon = e, eps
        run(M, m, A, b, P, op, 600)
        assert np.array_equal(P.qtable(), op.q)
    q = P.qtable()
    G = M.Policy(kind=M.POLICY_QTABLE, decision_period=D, per_op=1)
    G.set_qtable(q)
    run(M, m, A, b, G, O.OraclePolicy(kind=O.POL_QTABLE, q=q, decision_period=D, per_op=1), 2000)
    rng = np.random.default_rng(3)
    k = rng.integers(0, 3000, 500)
    rho = 10.0 ** rng.uniform(-17, 1, 500)
    stag = rng.integers(0, 2, 500)
    st, ac = G.decide(k, rho, stag)
    opg = O.OraclePolicy(kind=O.POL_QTABLE, q=q, per_op=1)
    for i in range(500):
        s = opg.state(int(k[i]), float(rho[i]), int(stag[i]))
        row = q[s]
        want = 16 * int(np.argmax(row[0:4])) + 4 * int(np.argmax(row[4:8])) + int(np.argmax(row[8:12]))
        assert st[i] == s and ac[i] == want
