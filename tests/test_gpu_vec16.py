"""16-bit vector storage on the GPU (vec16: bf16 updates keep r, p and x_lo in
bf16 containers), bit for bit against the oracle's vec16 mode: fixed actions
with bf16 updates and every other update format, tier changes into and out of
the bf16 containers under a Q-table, replacements, the fallback, and whole
solves at full size where the iteration runs from the 16-bit vectors."""
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


def run(M, m, A, b, pol, opol, tol=1e-8, maxit=3000, R=50, fallback=True):
    m.set_policy(pol)
    m.set_options(replace_period=R, fallback=fallback, vec16=1)
    xd = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    res = m.solve(torch.from_numpy(np.ascontiguousarray(b)).cuda(), xd, tol=tol, maxit=maxit)
    xo, info = O.cg(A, b, tol=tol, maxit=maxit, policy=opol, replace_period=R, fallback=fallback, vec16=1)
    assert_same(xd.cpu().numpy(), res, m.history(), xo, info)
    return res, info


ACTS = [(1, 2, 1), (1, 1, 1), (0, 0, 1), (2, 2, 1), (3, 3, 1), (5, 5, 1), (4, 2, 1), (1, 2, 2), (3, 3, 3), (0, 2, 0)]


@pytest.mark.parametrize("f", ACTS, ids=[f"{a}{b}{c}" for a, b, c in ACTS])
@pytest.mark.parametrize("A_fn", [lambda: W.laplacian_3d(20), lambda: W.random_spd(20001, 7, 1.5)],
                         ids=["lap3d_20", "rspd_20001"])
def test_fixed_actions_with_bf16_containers(M, A_fn, f):
    A = A_fn()
    b = W.rhs(A.n, 2)
    act = O.action(*f) if f[0] != 4 else 64 + 4 * f[1] + f[2]
    run(M, M.Matrix(A), A, b, M.Policy(kind=M.POLICY_FIXED, fixed_action=act), O.OraclePolicy(fixed_action=act))


def test_tier_changes_under_a_qtable(M):
    """A greedy table whose action alternates between bf16, fp32 and fp64
    updates with the residual bin: the containers change in both directions."""
    A = W.laplacian_2d(90)
    b = W.rhs(A.n, 5)
    rng = np.random.default_rng(3)
    q = rng.standard_normal((100, 64))
    for s in range(100):
        j = (s // 10) % 3
        q[s, [16 + 8 + 1, 16 + 8 + 2, 16 + 8 + 3][j]] += 100.0
    P = M.Policy(kind=M.POLICY_QTABLE)
    P.set_qtable(q)
    res, info = run(M, M.Matrix(A), A, b, P, O.OraclePolicy(kind=O.POL_QTABLE, q=q), maxit=4000, R=30)
    fl = info["flags"][:info["iters"]]
    assert np.count_nonzero(fl & O.FL_SWITCH) >= 2


def test_full_size_laplacian_bf16_updates(M):
    """3D Laplacian 128^3, bf16 SpMV and dots, bf16 updates from the 16-bit
    containers: 60 iterations (one replacement) against the oracle."""
    A = W.laplacian_3d(128)
    b = W.rhs(A.n, 2)
    act = O.action(1, 1, 1)
    run(M, M.Matrix(A), A, b, M.Policy(kind=M.POLICY_FIXED, fixed_action=act), O.OraclePolicy(fixed_action=act),
        maxit=60, fallback=False)


def test_vec16_refusals(M):
    A = W.laplacian_2d(16)
    m = M.Matrix(A)
    for kw in ({"precond": 1}, {"rho_fp64": 1}, {"emulate": 1}):
        with pytest.raises(M.MPCGError):
            m.set_options(vec16=1, **kw)
    m.set_options(vec16=1)
    m.set_policy(M.Policy(kind=M.POLICY_FIXED, fixed_action=21))
    b = torch.from_numpy(W.rhs(A.n, 1)).cuda()
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    with pytest.raises(M.MPCGError):
        M.solve_batched([(m, b, x)], tol=1e-8, maxit=100)
