"""Whole solves at the benchmark's full sizes, in its launch configuration, equal
the oracle's (section 3's recurrences at section 4.2's precisions: SpMV in bf16
storage with fp32 accumulation, dots and updates in fp32, fp64 replacement
every 50 iterations): status, iteration count, replacement log, the whole
residual history, the actions and the solution x, bit for bit.  The oracle's
results come from tests/golden/make_full_size_goldens.py (it calls only the
oracle); here the GPU side is compared with them through hashes of the arrays.
Also full SpMVs in fp16 and fp32 storage against the oracle's SpMV."""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def M():
    import paper_2504_14268_amd as M

    M.lib()
    assert torch.cuda.is_available()
    return M


def system(name):
    if name == "lap3d_128":
        A = W.laplacian_3d(128)
        return A, W.rhs(A.n, 2)
    A = W.random_spd(1_000_000, 3, W.spread_for_kappa(1e6))
    return A, W.rhs(A.n, 4)


def sha(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


@pytest.mark.parametrize("name", ["lap3d_128", "rspd_1e6"])
def test_full_size_whole_solve_equals_oracle(M, name):
    path = os.path.join(GOLD, f"full_size_{name}.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not written yet (tests/golden/make_full_size_goldens.py {name})")
    g = json.load(open(path))
    A, b = system(name)
    assert (A.n, A.nnz) == (g["n"], g["nnz"])
    m = M.Matrix(A)
    m.set_policy(M.Policy(kind=M.POLICY_FIXED, fixed_action=g["action"]))
    m.set_options(replace_period=g["replace_period"], fallback=g["fallback"])
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    res = m.solve(torch.from_numpy(b).cuda(), x, tol=g["tol"], maxit=g["maxit"])
    h = m.history()
    k = res["iters"]
    print(f"{name}: GPU {res['status']} {k} it relres {res['relres_true']:.3e}; oracle {g['status']} {g['iters']} it")
    assert res["status"] == g["status"] == 0 and k == g["iters"]
    assert res["n_replace"] == g["n_replace"] and res["fallback_at"] == g["fallback_at"]
    assert res["relres_true"].hex() == g["relres_true"] and res["relres_true"] <= g["tol"]
    nr = res["n_replace"]
    assert h["rep_k"][:nr].tolist() == g["rep_k"]
    assert [float(v).hex() for v in h["rep_rho"][:nr]] == g["rep_rho"]
    assert sha(h["rho"][:k + 1].astype(np.float64)) == g["sha256_rho"]
    assert sha(h["actions"][:k].astype(np.uint8)) == g["sha256_actions"]
    assert sha(x.cpu().numpy().astype(np.float64)) == g["sha256_x"]


@pytest.mark.parametrize("name", ["lap3d_128", "rspd_1e6"])
def test_full_size_spmv_fp16_fp32(M, name):
    A, _ = system(name)
    m = M.Matrix(A)
    p = np.random.default_rng(6).standard_normal(A.n).astype(np.float32)
    pd = torch.from_numpy(p).cuda()
    q = torch.empty(A.n, dtype=torch.float32, device="cuda")
    for f in (M.FP16, M.FP32):
        m.op_spmv(f, 0, pd, q)
        want = O.spmv(A, p.astype(np.float64), f, False).astype(np.float32)
        assert np.array_equal(q.cpu().numpy(), want), f
