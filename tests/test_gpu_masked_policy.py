"""Learned policies restricted to the SpMV format (the labelled "SpMV only"
variation of the experiments): a Q-table whose other actions hold -1e300 and a
network whose output bias holds -2^100 for them.  The restricted decision
path equals the oracle's bit for bit, and every action taken has fp32 dots
and updates (before a fallback)."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from test_gpu_solve import assert_same, gpu_solve  # noqa: E402
from test_oracle_policy import mlp_weights  # noqa: E402

KEEP = [O.action(fs, O.F32, O.F32) for fs in (O.F16, O.BF16, O.F32, O.F64)]
MASKED = np.array([a not in KEEP for a in range(64)])


@pytest.fixture(scope="module")
def M():
    import paper_2504_14268_amd as M

    M.lib()
    assert torch.cuda.is_available()
    return M


def check_actions(h, res):
    k = res["iters"] if res["fallback_at"] < 0 else res["fallback_at"]
    assert np.all(np.isin(h["actions"][:k], KEEP))


@pytest.mark.parametrize("A_fn", [lambda: W.laplacian_2d(90), lambda: W.random_spd(20000, 31, 0.5)],
                         ids=["lap2d_90", "rspd_20000"])
def test_masked_qtable(M, A_fn):
    A = A_fn()
    b = W.rhs(A.n, 4)
    q = np.random.default_rng(8).standard_normal((100, 64))
    q[:, MASKED] = -1e300
    P = M.Policy(kind=M.POLICY_QTABLE)
    P.set_qtable(q)
    x, res, h = gpu_solve(M, A, b, maxit=3000, policy=P, R=50, fallback=True)
    xo, info = O.cg(A, b, tol=1e-8, maxit=3000, policy=O.OraclePolicy(kind=O.POL_QTABLE, q=q), replace_period=50,
                    fallback=True)
    assert_same(x, res, h, xo, info)
    check_actions(h, res)
    assert len(set(h["actions"][:res["iters"]].tolist())) > 1


def test_masked_network(M):
    w = mlp_weights(5)
    w["b3"] = w["b3"].copy()
    w["b3"][MASKED] = np.float32(-2.0 ** 100)
    A = W.random_spd(5000, 17, 1.0)
    b = W.rhs(A.n, 18)
    P = M.Policy(kind=M.POLICY_MLP)
    P.set_mlp(w)
    x, res, h = gpu_solve(M, A, b, maxit=800, policy=P, R=50, fallback=True)
    xo, info = O.cg(A, b, tol=1e-8, maxit=800, policy=O.OraclePolicy(kind=O.POL_MLP, mlp=w), replace_period=50,
                    fallback=True)
    assert_same(x, res, h, xo, info)
    check_actions(h, res)
