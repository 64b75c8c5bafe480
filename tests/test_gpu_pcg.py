"""GPU parity of the Jacobi-preconditioned solve (section 3 with M = diag(A),
section 4.2's fixed-fp32 preconditioner) through the C ABI: the stored
inverse diagonal, and whole solves -- fixed actions in every format (q52
storage included), replacements with and without the direction restart, tier
switches of a greedy Q-table, the network policy, Q-learning episodes and the
fp64 fallback -- equal the oracle's bit for bit, at small sizes and at the
benchmark's full random-SPD size."""
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


def solve_pair(M, A, b, act=None, policy=None, opolicy=None, maxit=3000, R=50, fallback=False, m=None):
    m = m or M.Matrix(A)
    P = policy if policy is not None else M.Policy(kind=M.POLICY_FIXED, fixed_action=act)
    m.set_policy(P)
    m.set_options(replace_period=R, fallback=fallback, precond=1)
    bd = torch.from_numpy(np.ascontiguousarray(b)).cuda()
    xd = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    res = m.solve(bd, xd, tol=1e-8, maxit=maxit)
    h = m.history()
    op = opolicy if opolicy is not None else O.OraclePolicy(fixed_action=act)
    xo, info = O.cg(A, b, tol=1e-8, maxit=maxit, policy=op, replace_period=R, fallback=fallback, precond=1)
    return xd.cpu().numpy(), res, h, xo, info


def assert_same(x, res, h, xo, info):
    assert res["status"] == info["status"], (res, info["status"])
    assert res["iters"] == info["iters"] and res["n_replace"] == info["n_replace"]
    assert res["fallback_at"] == info["fallback_at"]
    k, nr = info["iters"], info["n_replace"]
    assert np.array_equal(h["rho"][:k + 1], info["rho"][:k + 1], equal_nan=True)
    assert np.array_equal(h["actions"][:k], info["actions"][:k])
    assert np.array_equal(h["flags"][:k], info["flags"][:k])
    assert np.array_equal(h["rep_k"][:nr], info["rep_k"][:nr])
    assert np.array_equal(h["rep_rho"][:nr], info["rep_rho"][:nr], equal_nan=True)
    assert res["relres_true"] == info["relres_true"] and res["cost_sum"] == info["cost_sum"]
    assert np.array_equal(x, xo)


MATS = {
    "rspd_20000_k1e8": lambda: W.random_spd(20000, 5, W.spread_for_kappa(1e8)),
    "lap3d_24": lambda: W.laplacian_3d(24),
    "band_20000": lambda: W.banded_spd(20000, 7, 4, spread=2.0),
}


@pytest.mark.parametrize("name", list(MATS))
def test_jacobi_inverse_bit_exact(M, name):
    A = MATS[name]()
    assert np.array_equal(M.Matrix(A).precond_inverse(), O.jacobi_inverse(A))


@pytest.mark.parametrize("name", list(MATS))
@pytest.mark.parametrize("act", [63, 42, 26, 10, 21, 74, 16 * 3 + 4 * 1 + 2])
def test_pcg_fixed_actions(M, name, act):
    A = MATS[name]()
    b = W.rhs(A.n, 4)
    x, res, h, xo, info = solve_pair(M, A, b, act=act, R=50 if act != 63 else 0, fallback=True)
    assert_same(x, res, h, xo, info)
    assert res["status"] in (0, 2) and res["relres_true"] <= 1e-8


def test_pcg_greedy_qtable_switches_tiers(M):
    rng = np.random.default_rng(12)
    q = rng.standard_normal((100, 64))
    A = W.random_spd(30000, 21, W.spread_for_kappa(1e6))
    b = W.rhs(A.n, 22)
    P = M.Policy(kind=M.POLICY_QTABLE)
    P.set_qtable(q)
    x, res, h, xo, info = solve_pair(M, A, b, policy=P, opolicy=O.OraclePolicy(kind=O.POL_QTABLE, q=q),
                                     maxit=2000, fallback=True)
    assert_same(x, res, h, xo, info)
    assert np.any(info["flags"] & O.FL_SWITCH)


def test_pcg_mlp_policy(M):
    from test_oracle_policy import mlp_weights

    w = mlp_weights(8)
    A = W.random_spd(12000, 23, W.spread_for_kappa(1e5))
    b = W.rhs(A.n, 24)
    P = M.Policy(kind=M.POLICY_MLP)
    P.set_mlp(w)
    x, res, h, xo, info = solve_pair(M, A, b, policy=P, opolicy=O.OraclePolicy(kind=O.POL_MLP, mlp=w),
                                     maxit=1500, fallback=True)
    assert_same(x, res, h, xo, info)


def test_pcg_qlearning_episodes(M):
    A = W.random_spd(8000, 25, W.spread_for_kappa(1e6))
    b = W.rhs(A.n, 26)
    P = M.Policy(kind=M.POLICY_QTABLE_TRAIN, cost="C2", seed=5)
    op = O.OraclePolicy(kind=O.POL_QTRAIN, cost="C2", seed=5)
    m = M.Matrix(A)
    for e in (1, 2, 3):
        eps = 1.0 - 0.45 * (e - 1)
        P.set_episode(e, eps)
        op.s.episode, op.s.epsilon = e, eps
        x, res, h, xo, info = solve_pair(M, A, b, policy=P, opolicy=op, maxit=400, fallback=True, m=m)
        assert_same(x, res, h, xo, info)
        assert np.array_equal(P.qtable(), op.q)


def test_pcg_full_size_random_spd(M):
    """The benchmark's random SPD (n = 1e6, about 18M entries, kappa about 1e6),
    mixed action with Jacobi: the whole solve equals the oracle's."""
    A = W.random_spd(1_000_000, 3, W.spread_for_kappa(1e6))
    b = W.rhs(A.n, 4)
    x, res, h, xo, info = solve_pair(M, A, b, act=M.action(M.BF16, M.FP32, M.FP32), maxit=2000)
    assert_same(x, res, h, xo, info)
    assert res["status"] == 0 and res["iters"] < 200


def test_batched_refuses_preconditioner(M):
    A = W.laplacian_2d(20)
    m = M.Matrix(A)
    m.set_options(replace_period=50, precond=1)
    b = torch.from_numpy(W.rhs(A.n, 1)).cuda()
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    with pytest.raises(M.MPCGError):
        M.solve_batched([(m, b, x)])
