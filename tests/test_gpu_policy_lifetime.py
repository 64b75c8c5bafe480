"""Policy lifetime on the GPU: a policy destroyed while a matrix still holds
it is detached from that matrix, whose next solve runs its default policy
(fixed fp64), bit for bit against the oracle's fp64 solve."""
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


def test_destroyed_policy_detaches(M):
    """Destroying a policy that a matrix still holds detaches it: the next
    solve runs the matrix's default policy (fixed fp64), as the oracle's fp64
    solve does, instead of reading freed memory."""
    A = W.laplacian_2d(24)
    b = W.rhs(A.n, 3)
    m = M.Matrix(A)
    P = M.Policy(kind=M.POLICY_QTABLE)
    P.set_qtable(np.random.default_rng(1).standard_normal((100, 64)))
    m.set_policy(P)
    m.set_options(replace_period=0, fallback=False)
    P.close()
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    res = m.solve(torch.from_numpy(b).cuda(), x, tol=1e-8, maxit=1000)
    xo, info = O.cg(A, b, tol=1e-8, maxit=1000)
    assert_same(x.cpu().numpy(), res, m.history(), xo, info)
    assert np.all(m.history()["actions"] == 63)
