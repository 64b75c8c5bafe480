"""GPU parity of whole solves through the C ABI against the oracle: iterates,
residual histories, actions, replacement logs, Q-tables and rollouts must be
bit-identical (same definitions and summation trees on both sides); status and
iteration counts equal.  Edge and failure cases included."""
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


def gpu_solve(M, A, b, x0=None, tol=1e-8, maxit=1000, policy=None, R=50, fallback=False, m=None):
    m = m or M.Matrix(A)
    m.set_policy(policy)
    m.set_options(replace_period=R, fallback=fallback)
    bd = torch.from_numpy(np.ascontiguousarray(b, dtype=np.float64)).cuda()
    xd = torch.zeros(A.n, dtype=torch.float64, device="cuda") if x0 is None else \
        torch.from_numpy(np.ascontiguousarray(x0, dtype=np.float64)).cuda()
    res = m.solve(bd, xd, tol=tol, maxit=maxit)
    h = m.history()
    return xd.cpu().numpy(), res, h


def assert_same(x, res, h, xo, info, check_x=True):
    assert res["status"] == info["status"], (res, info["status"])
    assert res["iters"] == info["iters"]
    assert res["n_replace"] == info["n_replace"]
    assert res["fallback_at"] == info["fallback_at"]
    k = info["iters"]
    assert np.array_equal(h["rho"][:k + 1], info["rho"][:k + 1], equal_nan=True)
    assert np.array_equal(h["actions"][:k], info["actions"][:k])
    assert np.array_equal(h["flags"][:k], info["flags"][:k])
    nr = info["n_replace"]
    assert np.array_equal(h["rep_k"][:nr], info["rep_k"][:nr])
    assert np.array_equal(h["rep_rho"][:nr], info["rep_rho"][:nr], equal_nan=True)
    assert res["relres_true"] == info["relres_true"] or (np.isnan(res["relres_true"]) and np.isnan(info["relres_true"]))
    assert res["cost_sum"] == info["cost_sum"]
    if check_x:
        assert np.array_equal(x, xo)


def test_fp64_cg_laplacian2d_64(M):
    """2D Laplacian 64x64, plain fp64 CG, tol 1e-8, maxit 2000, replacement only on the trigger."""
    A = W.laplacian_2d(64)
    b = W.rhs(A.n, 1)
    x, res, h = gpu_solve(M, A, b, maxit=2000, R=0)
    xo, info = O.cg(A, b, tol=1e-8, maxit=2000)
    assert res["status"] == 0 and res["relres_true"] <= 1e-8
    assert_same(x, res, h, xo, info)
    # after a fixed iteration count the fp64 iterate agrees to 1e-10 (here: exactly)
    x100, r100, _ = gpu_solve(M, A, b, maxit=100, R=0)
    xo100, i100 = O.cg(A, b, tol=1e-8, maxit=100)
    assert r100["status"] == 1
    assert np.linalg.norm(x100 - xo100) <= 1e-10 * np.linalg.norm(xo100)


@pytest.mark.parametrize("A_fn", [lambda: W.laplacian_3d(24), lambda: W.random_spd(20000, 7, 1.5)],
                         ids=["lap3d_24", "rspd_20000"])
@pytest.mark.parametrize("act", [0 * 16 + 2 * 4 + 2, 1 * 16 + 2 * 4 + 2, 2 * 16 + 2 * 4 + 2, 63,
                                 4 * 16 + 2 * 4 + 2])
def test_fixed_mixed(M, A_fn, act):
    A = A_fn()
    b = W.rhs(A.n, 2)
    P = M.Policy(kind=M.POLICY_FIXED, fixed_action=act)
    fb = act >= 64       # q52 storage (u = 1/8) stagnates on the scaled random SPD: fp64 fallback
    x, res, h = gpu_solve(M, A, b, maxit=6000, policy=P, R=50, fallback=fb)
    xo, info = O.cg(A, b, tol=1e-8, maxit=6000, policy=O.OraclePolicy(fixed_action=act), replace_period=50,
                    fallback=fb)
    assert_same(x, res, h, xo, info)
    assert res["status"] in ((0, 2) if fb else (0,)) and res["relres_true"] <= 1e-8
    r = O.residual(A, b, x)
    assert np.linalg.norm(r) / np.linalg.norm(b) <= 1e-8


def test_all_80_actions(M):
    """The 64 actions over the four arithmetic formats and the 16 with q52 SpMV storage."""
    A = W.random_spd(3000, 11, 2.0)
    b = W.rhs(A.n, 12)
    m = M.Matrix(A)
    for act in range(80):
        P = M.Policy(kind=M.POLICY_FIXED, fixed_action=act)
        x, res, h = gpu_solve(M, A, b, maxit=400, policy=P, R=50, fallback=(act % 2 == 0), m=m)
        xo, info = O.cg(A, b, tol=1e-8, maxit=400, policy=O.OraclePolicy(fixed_action=act),
                        replace_period=50, fallback=(act % 2 == 0))
        assert_same(x, res, h, xo, info)


def test_qtable_greedy_switching(M):
    rng = np.random.default_rng(4)
    q = rng.standard_normal((100, 64))
    A = W.random_spd(6000, 13, 1.0)
    b = W.rhs(A.n, 14)
    P = M.Policy(kind=M.POLICY_QTABLE)
    P.set_qtable(q)
    x, res, h = gpu_solve(M, A, b, maxit=1500, policy=P, R=50, fallback=True)
    xo, info = O.cg(A, b, tol=1e-8, maxit=1500, policy=O.OraclePolicy(kind=O.POL_QTABLE, q=q),
                    replace_period=50, fallback=True)
    assert_same(x, res, h, xo, info)
    assert len(set(info["actions"].tolist())) > 3


@pytest.mark.parametrize("cost", ["C1", "C2"])
def test_qlearning_training_episodes(M, cost):
    """Algorithm 1 on the device: epsilon-greedy draws, rewards and Q updates give
    the oracle's Q-table bit for bit after every episode; rollouts too."""
    A = W.laplacian_2d(40)
    b = W.rhs(A.n, 3)
    E = 4
    P = M.Policy(kind=M.POLICY_QTABLE_TRAIN, cost=cost, seed=77)
    P.rollouts_enable(20000)
    op = O.OraclePolicy(kind=O.POL_QTRAIN, cost=cost, seed=77)
    m = M.Matrix(A)
    all_roll = []
    for e in range(1, E + 1):
        eps = 1.0 - 0.9 * (e - 1) / (E - 1)
        P.set_episode(e, eps)
        op.s.episode, op.s.epsilon = e, eps
        x, res, h = gpu_solve(M, A, b, maxit=300, policy=P, R=50, fallback=True, m=m)
        xo, info = O.cg(A, b, tol=1e-8, maxit=300, policy=op, replace_period=50, fallback=True, roll_cap=5000)
        assert_same(x, res, h, xo, info)
        assert np.array_equal(P.qtable(), op.q)
        all_roll.append(info["rollouts"])
    g = P.rollouts()
    for key in ("feat", "next", "act", "rew", "done"):
        assert np.array_equal(g[key], np.concatenate([r[key] for r in all_roll]))


@pytest.mark.parametrize("kind", ["qtable", "mlp"])
def test_logging_policies_full_step(M, kind):
    """Policies that only read shared state (a fixed Q-table, the network) with
    rollout logging run the full step in every KB workgroup and log from
    workgroup 0: 20,000 rows (10 vector blocks, a ragged tail); both policies
    stagnate, fall back to fp64 and converge, which logs a terminal row.
    The solve and the logged rollouts equal the oracle's bit for bit."""
    from test_oracle_policy import mlp_weights

    A = W.random_spd(20000, 31, 0.5)
    b = W.rhs(A.n, 32)
    if kind == "qtable":
        q = np.random.default_rng(6).standard_normal((100, 64))
        P = M.Policy(kind=M.POLICY_QTABLE)
        P.set_qtable(q)
        op = O.OraclePolicy(kind=O.POL_QTABLE, q=q)
    else:
        w = mlp_weights(7)
        P = M.Policy(kind=M.POLICY_MLP)
        P.set_mlp(w)
        op = O.OraclePolicy(kind=O.POL_MLP, mlp=w)
    P.rollouts_enable(5000)
    x, res, h = gpu_solve(M, A, b, maxit=700, policy=P, R=50, fallback=True)
    xo, info = O.cg(A, b, tol=1e-8, maxit=700, policy=op, replace_period=50, fallback=True, roll_cap=5000)
    assert_same(x, res, h, xo, info)
    assert res["status"] == 2
    g = P.rollouts()
    assert len(g["act"]) == len(info["rollouts"]["act"]) > 10
    for key in ("feat", "next", "act", "rew", "done"):
        assert np.array_equal(g[key], info["rollouts"][key]), key


def test_mlp_policy_solve(M):
    from test_oracle_policy import mlp_weights

    w = mlp_weights(5)
    A = W.random_spd(5000, 17, 1.0)
    b = W.rhs(A.n, 18)
    P = M.Policy(kind=M.POLICY_MLP)
    P.set_mlp(w)
    x, res, h = gpu_solve(M, A, b, maxit=800, policy=P, R=50, fallback=True)
    xo, info = O.cg(A, b, tol=1e-8, maxit=800, policy=O.OraclePolicy(kind=O.POL_MLP, mlp=w),
                    replace_period=50, fallback=True)
    assert_same(x, res, h, xo, info)


def test_edge_cases(M):
    A = W.laplacian_2d(10)
    b = W.rhs(A.n, 1)
    x, res, h = gpu_solve(M, A, b, maxit=0)
    assert res["status"] == 1 and res["iters"] == 0
    x, res, h = gpu_solve(M, A, np.zeros(A.n), x0=np.ones(A.n), maxit=10)
    assert res["status"] == 0 and np.all(x == 0)
    xs = np.linalg.solve(A.to_dense(), b)
    x, res, h = gpu_solve(M, A, b, x0=xs, maxit=10)
    xo, info = O.cg(A, b, x0=xs, maxit=10)
    assert res["status"] == 0 and res["iters"] == 0 and np.array_equal(x, xo)
    bn = b.copy()
    bn[3] = np.nan
    x, res, h = gpu_solve(M, A, bn, maxit=10)
    assert res["status"] == 3
    # 1x1 system and a tiny ragged one
    A1 = W.CSR(1, np.array([0, 1], np.int32), np.array([0], np.int32), np.array([4.0]))
    x, res, h = gpu_solve(M, A1, np.array([2.0]), maxit=5)
    assert res["status"] == 0 and x[0] == 0.5


def test_indefinite_and_fp16_hostile(M):
    A = W.laplacian_2d(10)
    A.val = A.val.copy()
    diag = A.col == np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    A.val[diag] = -4.0
    with pytest.raises(M.MPCGError):       # the boundary rejects a non-positive diagonal
        M.Matrix(A)
    A = W.random_spd(2000, 31, spread=3.0)
    b = W.rhs(A.n, 32) * 1e6
    for fb in (True, False):
        P = M.Policy(kind=M.POLICY_FIXED, fixed_action=0)
        x, res, h = gpu_solve(M, A, b, maxit=20000, policy=P, R=50, fallback=fb)
        xo, info = O.cg(A, b, tol=1e-8, maxit=20000, policy=O.OraclePolicy(fixed_action=0),
                        replace_period=50, fallback=fb)
        assert_same(x, res, h, xo, info)
    assert info["status"] in (1, 3)


def test_run_twice_identical(M):
    A = W.random_spd(30000, 21, 1.5)
    b = W.rhs(A.n, 22)
    P = M.Policy(kind=M.POLICY_FIXED, fixed_action=1 * 16 + 2 * 4 + 2)
    m = M.Matrix(A)
    x1, r1, h1 = gpu_solve(M, A, b, maxit=4000, policy=P, m=m)
    x2, r2, h2 = gpu_solve(M, A, b, maxit=4000, policy=P, m=m)
    assert np.array_equal(x1, x2) and np.array_equal(h1["rho"], h2["rho"])
    r1.pop("time_ms"); r2.pop("time_ms")
    assert r1 == r2


def test_index16_equals_index32(M):
    """16-bit column deltas change only the bytes read: same history and x."""
    import torch

    A = W.laplacian_3d(24)
    b = W.rhs(A.n, 8)
    m = M.Matrix(A)
    assert m.info()["index16"]
    assert not M.Matrix(W.random_spd(70000, 3, 1.0)).info()["index16"]
    out = []
    for idx in (0, -1):
        m.set_policy(M.Policy(kind=M.POLICY_FIXED, fixed_action=M.action(M.FP16, M.FP32, M.FP32)))
        m.set_options(replace_period=50, fallback=False, index16=idx)
        x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        r = m.solve(torch.from_numpy(b).cuda(), x, tol=1e-8, maxit=500)
        out.append((r, x.cpu().numpy(), m.history()))
    (r1, x1, h1), (r2, x2, h2) = out
    assert r1["iters"] == r2["iters"] and np.array_equal(x1, x2) and np.array_equal(h1["rho"], h2["rho"])
    xo, info = O.cg(A, b, tol=1e-8, maxit=500, policy=O.OraclePolicy(fixed_action=M.action(M.FP16, M.FP32, M.FP32)),
                    replace_period=50)
    assert_same(x1, r1, h1, xo, info)


@pytest.mark.parametrize("which", ["lap3d_128", "rspd_1M"])
def test_full_size_first_iterations(M, which):
    """At the benchmark's full sizes and launch configuration: the first
    iterations (start, three CG steps, final true residual) equal the oracle's
    bit for bit, and a full SpMV in the benchmark's format matches too."""
    import torch

    if which == "lap3d_128":
        A, b = W.laplacian_3d(128), W.rhs(128 ** 3, 2)
    else:
        A = W.random_spd(1_000_000, 3, W.spread_for_kappa(1e6))
        b = W.rhs(A.n, 4)
    act = M.action(M.BF16, M.FP32, M.FP32)
    x, res, h = gpu_solve(M, A, b, maxit=3, policy=M.Policy(kind=M.POLICY_FIXED, fixed_action=act), R=50)
    xo, info = O.cg(A, b, tol=1e-8, maxit=3, policy=O.OraclePolicy(fixed_action=act), replace_period=50)
    assert_same(x, res, h, xo, info)
    m = M.Matrix(A)
    p = np.random.default_rng(5).standard_normal(A.n).astype(np.float32)
    q = torch.empty(A.n, dtype=torch.float32, device="cuda")
    # the benchmark's bf16 storage, and fp16 and q52 with their row scales
    for fmt in (M.BF16, M.FP16, M.Q52):
        m.op_spmv(fmt, 0, torch.from_numpy(p).cuda(), q)
        assert np.array_equal(q.cpu().numpy(), O.spmv(A, p.astype(np.float64), fmt, False).astype(np.float32)), fmt
