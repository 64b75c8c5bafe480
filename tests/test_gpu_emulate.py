"""The paper's emulation reading on the GPU (emulate = 1: fp64 operations whose
results are rounded to the operation's format, fp64 vectors), bit for bit
against the oracle's emulation mode: fixed actions over the five arithmetic
formats, with the Jacobi preconditioner and fp64 rho, and Q-learning in the
paper's setting (section 5)."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from test_gpu_solve import assert_same  # noqa: E402


@pytest.fixture(scope="module")
def M():
    import paper_2504_14268_amd as M

    M.lib()
    assert torch.cuda.is_available()
    return M


def solve_both(M, m, A, b, act_or_pol, opol, tol, maxit, **opts):
    pol = act_or_pol if not isinstance(act_or_pol, int) else M.Policy(kind=M.POLICY_FIXED, fixed_action=act_or_pol)
    m.set_policy(pol)
    m.set_options(emulate=1, **opts)
    xd = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    res = m.solve(torch.from_numpy(np.ascontiguousarray(b)).cuda(), xd, tol=tol, maxit=maxit)
    oo = dict(opts)
    R = oo.pop("replace_period", 50)
    xo, info = O.cg(A, b, tol=tol, maxit=maxit, policy=opol, replace_period=R, emulate=1, **oo)
    assert_same(xd.cpu().numpy(), res, m.history(), xo, info)
    return res, info


F = [O.F16, O.BF16, O.F32, O.F64, O.TF32]
ACTS = [(1, 3, 3), (0, 3, 3), (5, 3, 3), (2, 2, 2), (3, 1, 3), (3, 0, 3), (3, 5, 3), (3, 3, 1), (3, 3, 5),
        (1, 1, 1), (5, 5, 5), (2, 1, 5)]


@pytest.mark.parametrize("f", ACTS, ids=[f"{a}{b}{c}" for a, b, c in ACTS])
@pytest.mark.parametrize("A_fn", [lambda: W.laplacian_3d(20), lambda: W.random_spd(20000, 7, 1.5)],
                         ids=["lap3d_20", "rspd_20000"])
def test_fixed_actions_emulated(M, A_fn, f):
    A = A_fn()
    b = W.rhs(A.n, 2)
    act = O.action(*f)
    res, info = solve_both(M, M.Matrix(A), A, b, act, O.OraclePolicy(fixed_action=act), 1e-8, 3000,
                           replace_period=50, fallback=True)
    assert res["status"] in (0, 1, 2)


@pytest.mark.parametrize("precond,rho64", [(1, 0), (0, 1), (1, 1)])
def test_emulated_with_preconditioner_and_fp64_rho(M, precond, rho64):
    A = W.random_spd(30000, 9, 2.0)
    b = W.rhs(A.n, 3)
    m = M.Matrix(A)
    for f in [(1, 3, 3), (5, 1, 3), (2, 5, 1), (3, 3, 3)]:
        act = O.action(*f)
        solve_both(M, m, A, b, act, O.OraclePolicy(fixed_action=act), 1e-9, 3000, replace_period=40,
                   fallback=True, precond=precond, rho_fp64=rho64)


def test_emulated_paper_setting_qlearning(M):
    """Algorithm 1 in the paper's setting under its emulation reading: tables
    for SpMV and dot over five formats, updates in fp64, rho < 1e-6 with
    k >= 10, fp64 rho, epsilon from 1 down; the table after every episode."""
    A1 = W.bbt_system(7, density_reading="pairs")
    A2, b2 = W.poisson_subdomain(8)
    systems = [(A1, W.rhs(A1.n, 9)), (A2, b2)]
    P = M.Policy(kind=M.POLICY_QTABLE_TRAIN, cost="C1", seed=29, per_op=2, nfmt=5)
    op = O.OraclePolicy(kind=O.POL_QTRAIN, cost="C1", seed=29, per_op=2, nfmt=5)
    mats = [M.Matrix(A) for A, _ in systems]
    e = 0
    for sweep in range(3):
        for (A, b), m in zip(systems, mats):
            e += 1
            eps = 1.0 - 0.9 * (e - 1) / 5
            P.set_episode(e, eps)
            op.s.episode, op.s.epsilon = e, eps
            solve_both(M, m, A, b, P, op, 1e-6, 1000, replace_period=50, fallback=False, stop_rule=1, rho_fp64=1)
            assert np.array_equal(P.qtable(), op.q)


def test_emulation_refusals(M):
    A = W.laplacian_2d(16)
    m = M.Matrix(A)
    m.set_policy(M.Policy(kind=M.POLICY_FIXED, fixed_action=64 + 4 * 2 + 2))   # a q52 SpMV
    m.set_options(emulate=1)
    b = torch.from_numpy(W.rhs(A.n, 1)).cuda()
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    with pytest.raises(M.MPCGError):
        m.solve(b, x, tol=1e-8, maxit=100)
    m.set_policy(M.Policy(kind=M.POLICY_FIXED, fixed_action=21))
    with pytest.raises(M.MPCGError):
        M.solve_batched([(m, b, x)], tol=1e-8, maxit=100)
