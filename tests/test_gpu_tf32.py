"""tf32 on the GPU, bit for bit against the oracle: the action codes, whole
solves whose SpMV, dots or updates are in tf32 (emulated: values rounded to
tf32 and held in fp32 containers), with and without the Jacobi
preconditioner and fp64 rho, and Q-learning with one table per operation over
the paper's five formats {fp16, bf16, tf32, fp32, fp64} (section 5)."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from test_gpu_solve import assert_same, gpu_solve  # noqa: E402


@pytest.fixture(scope="module")
def M():
    import paper_2504_14268_amd as M

    M.lib()
    assert torch.cuda.is_available()
    return M


def test_action_codes_match_the_oracle(M):
    fmts = [M.FP16, M.BF16, M.FP32, M.FP64, M.TF32]
    for fs in fmts:
        for fd in fmts:
            for fa in fmts:
                a = M.action(fs, fd, fa)
                assert a == O.action(fs, fd, fa)
                assert M.decode(a) == O.act_decode(a) == (fs, fd, fa)
    for a in range(64, 80):
        assert M.decode(a) == O.act_decode(a)
    for bad in (80, 127, 253, -1):
        with pytest.raises(M.MPCGError):
            M.decode(bad)


TF32_ACTIONS = {
    "spmv": (5, 3, 3), "dot": (3, 5, 3), "update": (3, 3, 5), "all": (5, 5, 5),
    "spmv_dot_fp32_update": (5, 5, 2), "bf16_spmv_tf32_rest": (1, 5, 5),
}


@pytest.mark.parametrize("name", list(TF32_ACTIONS))
@pytest.mark.parametrize("A_fn", [lambda: W.laplacian_3d(20), lambda: W.random_spd(20000, 7, 1.5)],
                         ids=["lap3d_20", "rspd_20000"])
def test_fixed_tf32_solves(M, A_fn, name):
    A = A_fn()
    b = W.rhs(A.n, 2)
    act = O.action(*TF32_ACTIONS[name])
    x, res, h = gpu_solve(M, A, b, maxit=4000, policy=M.Policy(kind=M.POLICY_FIXED, fixed_action=act), R=50,
                          fallback=True)
    xo, info = O.cg(A, b, tol=1e-8, maxit=4000, policy=O.OraclePolicy(fixed_action=act), replace_period=50,
                    fallback=True)
    assert_same(x, res, h, xo, info)
    assert res["status"] in (0, 2)


@pytest.mark.parametrize("precond,rho64", [(1, 0), (0, 1), (1, 1)])
def test_tf32_with_preconditioner_and_fp64_rho(M, precond, rho64):
    A = W.random_spd(30000, 9, 2.0)
    b = W.rhs(A.n, 3)
    m = M.Matrix(A)
    for f in [(1, 5, 5), (5, 5, 2), (5, 0, 5)]:
        act = O.action(*f)
        m.set_policy(M.Policy(kind=M.POLICY_FIXED, fixed_action=act))
        m.set_options(replace_period=40, fallback=True, precond=precond, rho_fp64=rho64)
        xd = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        res = m.solve(torch.from_numpy(b).cuda(), xd, tol=1e-9, maxit=3000)
        h = m.history()
        xo, info = O.cg(A, b, tol=1e-9, maxit=3000, policy=O.OraclePolicy(fixed_action=act), replace_period=40,
                        fallback=True, precond=precond, rho_fp64=rho64)
        assert_same(xd.cpu().numpy(), res, h, xo, info)


@pytest.mark.parametrize("per_op", [1, 2])
def test_five_format_qlearning_bit_exact(M, per_op):
    """Episodes of Algorithm 1 with one table per operation over five formats,
    the paper's termination and fp64 rho, on the paper's two families; the
    Q-table after every episode and then the greedy solves."""
    A1 = W.bbt_system(7, density_reading="pairs")
    A2, b2 = W.poisson_subdomain(8)
    systems = [(A1, W.rhs(A1.n, 9)), (A2, b2)]
    P = M.Policy(kind=M.POLICY_QTABLE_TRAIN, cost="C2", seed=23, per_op=per_op, nfmt=5)
    op = O.OraclePolicy(kind=O.POL_QTRAIN, cost="C2", seed=23, per_op=per_op, nfmt=5)
    mats = [M.Matrix(A) for A, _ in systems]

    def run(m, A, b, pol, opol):
        m.set_policy(pol)
        m.set_options(replace_period=50, fallback=False, stop_rule=1, rho_fp64=1)
        xd = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        res = m.solve(torch.from_numpy(np.ascontiguousarray(b)).cuda(), xd, tol=1e-6, maxit=1000)
        xo, info = O.cg(A, b, tol=1e-6, maxit=1000, policy=opol, replace_period=50, stop_rule=1, rho_fp64=1)
        assert_same(xd.cpu().numpy(), res, m.history(), xo, info)
        return info

    e = 0
    seen_tf32 = False
    for sweep in range(3):
        for (A, b), m in zip(systems, mats):
            e += 1
            eps = 1.0 - 0.9 * (e - 1) / 5
            P.set_episode(e, eps)
            op.s.episode, op.s.epsilon = e, eps
            info = run(m, A, b, P, op)
            assert np.array_equal(P.qtable(), op.q)
            seen_tf32 |= bool(np.any(info["actions"][:info["iters"]] >= 128))
    assert seen_tf32
    G = M.Policy(kind=M.POLICY_QTABLE, cost="C2", per_op=per_op, nfmt=5)
    G.set_qtable(P.qtable())
    for (A, b), m in zip(systems, mats):
        run(m, A, b, G, O.OraclePolicy(kind=O.POL_QTABLE, q=op.q, cost="C2", per_op=per_op, nfmt=5))


def test_tf32_refusals(M):
    with pytest.raises(M.MPCGError):
        M.Policy(kind=M.POLICY_QTABLE_TRAIN, nfmt=5)          # five formats need per-operation tables
    with pytest.raises(M.MPCGError):
        M.Policy(kind=M.POLICY_FIXED, fixed_action=100)       # not an action code
    A = W.laplacian_2d(16)
    m = M.Matrix(A)
    m.set_policy(M.Policy(kind=M.POLICY_FIXED, fixed_action=O.action(5, 3, 3)))
    b = torch.from_numpy(W.rhs(A.n, 1)).cuda()
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    with pytest.raises(M.MPCGError):
        M.solve_batched([(m, b, x)], tol=1e-8, maxit=100)
