"""The paper's own experimental setting on the GPU, bit for bit against the
oracle: the synthetic families of section 5 (A = B B^T + beta I with n = 5000,
and the 2D Poisson problem on a random subdomain, 80 x 80), section 5's
termination (the recursive residual below 1e-6 after at least 10
iterations), and Q-learning with one table per operation (section 4.1)."""
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


def systems():
    A1 = W.bbt_system(7, density_reading="pairs")
    A2, b2 = W.poisson_subdomain(8)
    return [(A1, W.rhs(A1.n, 9)), (A2, b2)]


def compare(M, m, A, b, P, op, maxit=1000, tol=1e-6, rho_fp64=0):
    m.set_policy(P)
    m.set_options(replace_period=50, fallback=False, stop_rule=1, rho_fp64=rho_fp64)
    xd = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    res = m.solve(torch.from_numpy(np.ascontiguousarray(b)).cuda(), xd, tol=tol, maxit=maxit)
    h = m.history()
    xo, info = O.cg(A, b, tol=tol, maxit=maxit, policy=op, replace_period=50, stop_rule=1, rho_fp64=rho_fp64)
    k = info["iters"]
    assert (res["status"], res["iters"]) == (info["status"], k)
    assert np.array_equal(h["rho"][:k + 1], info["rho"][:k + 1])
    assert np.array_equal(h["actions"][:k], info["actions"][:k])
    assert res["relres_true"] == info["relres_true"] and np.array_equal(xd.cpu().numpy(), xo)
    return res, info


@pytest.mark.parametrize("rho_fp64", [0, 1])
@pytest.mark.parametrize("act", [63, 16 * 1 + 4 * 2 + 2, 16 * 0 + 4 * 1 + 2, 16 * 0 + 4 * 0 + 3, 16 * 3 + 4 * 0 + 3])
def test_paper_termination_fixed_actions(M, act, rho_fp64):
    for A, b in systems():
        res, info = compare(M, M.Matrix(A), A, b, M.Policy(kind=M.POLICY_FIXED, fixed_action=act),
                            O.OraclePolicy(fixed_action=act), rho_fp64=rho_fp64)
        if res["status"] == 0:
            assert res["iters"] >= 10 and info["rho"][res["iters"]] < 1e-6


@pytest.mark.parametrize("per_op,rho_fp64", [(1, 0), (2, 0), (2, 1)])
def test_paper_setting_per_op_qlearning(M, per_op, rho_fp64):
    """Algorithm 1 as the paper runs it: one table per operation (per_op 2:
    SpMV and dot only, the updates in fp64), cost setting C2, tol 1e-6 with
    k >= 10, T_max 1000, epsilon from 1 down; then the greedy tables."""
    sys = systems()
    P = M.Policy(kind=M.POLICY_QTABLE_TRAIN, cost="C2", seed=21, per_op=per_op)
    op = O.OraclePolicy(kind=O.POL_QTRAIN, cost="C2", seed=21, per_op=per_op)
    mats = [M.Matrix(A) for A, _ in sys]
    e = 0
    for sweep in range(3):
        for (A, b), m in zip(sys, mats):
            e += 1
            eps = 1.0 - 0.9 * (e - 1) / 5
            P.set_episode(e, eps)
            op.s.episode, op.s.epsilon = e, eps
            compare(M, m, A, b, P, op, rho_fp64=rho_fp64)
            assert np.array_equal(P.qtable(), op.q)
    G = M.Policy(kind=M.POLICY_QTABLE, cost="C2", per_op=per_op)
    G.set_qtable(P.qtable())
    for (A, b), m in zip(sys, mats):
        res, info = compare(M, m, A, b, G, O.OraclePolicy(kind=O.POL_QTABLE, q=op.q, per_op=per_op),
                            rho_fp64=rho_fp64)
        if per_op == 2:
            assert np.all(info["actions"][:info["iters"]] & 3 == 3)


@pytest.mark.parametrize("precond", [0, 1])
def test_rho_fp64_with_and_without_preconditioner(M, precond):
    """rho from an fp64 r.r, sigma' (r.r or r.z) at the dot format: the default
    termination with replacements, fp16 and bf16 dots, Jacobi on and off."""
    A = W.laplacian_3d(20)
    b = W.rhs(A.n, 4)
    m = M.Matrix(A)
    for act in (16 * 1 + 4 * 0 + 2, 16 * 2 + 4 * 1 + 2, 16 * 0 + 4 * 0 + 3):
        m.set_policy(M.Policy(kind=M.POLICY_FIXED, fixed_action=act))
        m.set_options(replace_period=25, fallback=True, precond=precond, rho_fp64=1)
        xd = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        res = m.solve(torch.from_numpy(b).cuda(), xd, tol=1e-9, maxit=600)
        h = m.history()
        xo, info = O.cg(A, b, tol=1e-9, maxit=600, policy=O.OraclePolicy(fixed_action=act), replace_period=25,
                        fallback=True, precond=precond, rho_fp64=1)
        k = info["iters"]
        assert (res["status"], res["iters"]) == (info["status"], k), act
        assert np.array_equal(h["rho"][:k + 1], info["rho"][:k + 1]), act
        assert np.array_equal(xd.cpu().numpy(), xo), act
