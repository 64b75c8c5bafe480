"""Matrices created from device arrays (MPCG_MEM_DEVICE): the same shadows and
the same solve, bit for bit, as from host arrays; the same CSR validation
(the device arrays are copied to the host and checked the same way)."""
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


def dev(A):
    return (torch.from_numpy(np.ascontiguousarray(A.row_ptr, dtype=np.int32)).cuda(),
            torch.from_numpy(np.ascontiguousarray(A.col, dtype=np.int32)).cuda(),
            torch.from_numpy(np.ascontiguousarray(A.val, dtype=np.float64)).cuda())


@pytest.mark.parametrize("A_fn", [lambda: W.laplacian_3d(20), lambda: W.random_spd(20001, 7, 1.5)],
                         ids=["lap3d_20", "rspd_20001"])
def test_device_arrays_give_the_host_result(M, A_fn):
    A = A_fn()
    b = W.rhs(A.n, 2)
    mh = M.Matrix(A)
    md = M.Matrix.from_device(*dev(A))
    assert md.info() == mh.info()
    for u, v in zip(mh.shadows(), md.shadows()):
        assert np.array_equal(u, v)
    act = O.action(1, 2, 2)
    xo, info = O.cg(A, b, tol=1e-8, maxit=3000, replace_period=50, policy=O.OraclePolicy(fixed_action=act))
    for m in (mh, md):
        m.set_policy(M.Policy(kind=M.POLICY_FIXED, fixed_action=act))
        m.set_options(replace_period=50, fallback=False)
        x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        res = m.solve(torch.from_numpy(b).cuda(), x, tol=1e-8, maxit=3000)
        assert_same(x.cpu().numpy(), res, m.history(), xo, info)


def test_device_arrays_are_validated(M):
    A = W.laplacian_2d(12)
    rp, ci, v = dev(A)
    bad = ci.clone()
    bad[5] = A.n + 3                      # a column out of range
    with pytest.raises(M.MPCGError, match="row"):
        M.Matrix.from_device(rp, bad, v)
    nv = v.clone()
    nv[0] = float("nan")                  # a non-finite value
    with pytest.raises(M.MPCGError):
        M.Matrix.from_device(rp, ci, nv)
