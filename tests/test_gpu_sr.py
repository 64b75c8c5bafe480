"""Single-reduction CG (variant 1: Chronopoulos-Gear) and pipelined CG
(variant 2: Ghysels-Vanroose), two launches per iteration each, on the GPU,
bit for bit against the oracle's cg_sr and cg_pipe: status,
iterations, every rho_k, the actions and flags, the replacements, the true
relres and x.  Fixed actions over every SpMV format (q52 included), dot and
update format; a 3D Laplacian and a ragged random SPD that span several row
groups and vector blocks; a full-size 128^3 run through two replacements; the
degenerate cases; and the options the variant refuses."""
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


def run(M, m, A, b, act, tol=1e-8, maxit=3000, R=50, x0=None, spmv_rows=0, index16=0, variant=1):
    m.set_policy(M.Policy(kind=M.POLICY_FIXED, fixed_action=act))
    m.set_options(replace_period=R, fallback=False, variant=variant, spmv_rows=spmv_rows, index16=index16)
    x0 = np.zeros(A.n) if x0 is None else x0
    xd = torch.from_numpy(np.ascontiguousarray(x0, dtype=np.float64)).cuda()
    res = m.solve(torch.from_numpy(np.ascontiguousarray(b, dtype=np.float64)).cuda(), xd, tol=tol, maxit=maxit)
    cg = O.cg_sr if variant == 1 else O.cg_pipe
    xo, info = cg(A, b, act, x0=x0, tol=tol, maxit=maxit, replace_period=R)
    assert_same(xd.cpu().numpy(), res, m.history(), xo, info)
    return res, info


ACTS = [(1, 2, 2), (2, 2, 2), (3, 3, 3), (0, 2, 2), (1, 1, 2), (3, 3, 2), (2, 3, 3), (1, 0, 2), (1, 2, 1), (1, 2, 0)]


@pytest.mark.parametrize("variant", [1, 2], ids=["sr", "pipe"])
@pytest.mark.parametrize("f", ACTS + ["q52"], ids=[f"{a}{b}{c}" for a, b, c in ACTS] + ["q52"])
@pytest.mark.parametrize("A_fn", [lambda: W.laplacian_3d(20), lambda: W.random_spd(20001, 7, 1.5)],
                         ids=["lap3d_20", "rspd_20001"])
def test_fixed_actions_bit_exact(M, A_fn, f, variant):
    A = A_fn()
    b = W.rhs(A.n, 2)
    act = 64 + 4 * 2 + 2 if f == "q52" else O.action(*f)
    run(M, M.Matrix(A), A, b, act, R=50 if variant == 1 else 10, variant=variant)


@pytest.mark.parametrize("R", [0, 1, 7])
@pytest.mark.parametrize("rows", [512, 2048])
def test_replacement_periods_and_group_sizes(M, R, rows):
    """Replacement on the trigger only, after every iteration, every 7; the
    SpMV row groups of 512 and 2048 rows give the same bits.  Without periodic
    replacements the bf16 SpMV's recurrences drift until the step breaks down
    (iteration 461, after one triggered replacement), as in the oracle."""
    A = W.laplacian_2d(150)
    b = W.rhs(A.n, 3)
    res, info = run(M, M.Matrix(A), A, b, O.action(1, 2, 2), R=R, spmv_rows=rows)
    assert res["status"] == (3 if R == 0 else 0)
    run(M, M.Matrix(A), A, b, O.action(1, 2, 2), R=R, spmv_rows=rows, variant=2)


@pytest.mark.parametrize("variant", [1, 2], ids=["sr", "pipe"])
@pytest.mark.parametrize("f", [(1, 2, 2), (0, 2, 2), (3, 3, 3)], ids=["122", "022", "333"])
def test_int32_indices_and_initial_guess(M, f, variant):
    """The SpMV reading 32-bit column indices (index16 = -1) gives the same
    bits as the oracle, from a nonzero initial guess."""
    A = W.laplacian_3d(24)
    b = W.rhs(A.n, 8)
    x0 = np.random.default_rng(9).uniform(-1.0, 1.0, A.n)
    res, _ = run(M, M.Matrix(A), A, b, O.action(*f), x0=x0, index16=-1, R=10, variant=variant)
    assert res["index16"] == 0 and res["status"] == 0


def test_fp64_matches_the_three_launch_solver(M):
    """In fp64 the iterates are section 3's: the iteration count of the main
    solver (within one: the rounding of the recursive residual decides the
    iteration where it crosses tol) and x equal to rounding."""
    A = W.random_spd(30000, 5, 1.0)
    b = W.rhs(A.n, 4)
    m = M.Matrix(A)
    res, info = run(M, m, A, b, 63, tol=1e-10, R=0)
    m.set_options(replace_period=0, fallback=False)
    x2 = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    r2 = m.solve(torch.from_numpy(b).cuda(), x2, tol=1e-10, maxit=3000)
    xo, _ = O.cg_sr(A, b, 63, tol=1e-10, maxit=3000)
    assert r2["status"] == 0 and abs(res["iters"] - r2["iters"]) <= 1
    x2 = x2.cpu().numpy()
    assert np.abs(xo - x2).max() <= 1e-8 * np.abs(x2).max()


@pytest.mark.parametrize("variant", [1, 2], ids=["sr", "pipe"])
def test_full_size_laplacian(M, variant):
    """3D Laplacian 128^3 with the benchmark's mixed action: 45 iterations
    through two replacements (every 20), bit for bit."""
    A = W.laplacian_3d(128)
    b = W.rhs(A.n, 2)
    res, info = run(M, M.Matrix(A), A, b, O.action(1, 2, 2), maxit=45, R=20, variant=variant)
    assert res["status"] == 1 and res["iters"] == 45 and res["n_replace"] == 2


@pytest.mark.parametrize("variant", [1, 2], ids=["sr", "pipe"])
def test_degenerate_cases(M, variant):
    A = W.laplacian_2d(33)
    m = M.Matrix(A)
    act = O.action(1, 2, 2)
    res, _ = run(M, m, A, np.zeros(A.n), act, variant=variant)                 # b = 0: x = 0
    assert res["status"] == 0 and res["iters"] == 0
    xs = np.linalg.solve(A.to_dense(), W.rhs(A.n, 1))
    res, _ = run(M, m, A, A.to_dense() @ xs, act, x0=xs, variant=variant)      # exact initial guess
    assert res["status"] == 0 and res["iters"] == 0
    res, _ = run(M, m, A, W.rhs(A.n, 1), act, maxit=0, variant=variant)        # no iteration allowed
    assert res["status"] == 1 and res["iters"] == 0
    res, _ = run(M, m, A, W.rhs(A.n, 1), act, maxit=13, R=0, variant=variant)  # budget stop, no replacement
    assert res["status"] == 1 and res["iters"] == 13
    # indefinite with a positive diagonal: blocks [[1, 2], [2, 1]] (eigenvalues
    # 3 and -1) and b = (1, -1, ...): w = A b = -b, delta_0 = -||b||^2 < 0
    n = 8
    rows = np.repeat(np.arange(n), 2)
    cols = np.stack([np.arange(n), np.arange(n) ^ 1], axis=1).ravel()
    vals = np.tile([1.0, 2.0], n)
    D = W._from_coo(n, rows, cols, vals, "indef")
    mD = M.Matrix(D)
    res, info = run(M, mD, D, np.where(np.arange(n) % 2 == 0, 1.0, -1.0), 63, variant=variant)
    assert res["status"] == 3 and res["iters"] == 0
    # n = 3 and a few rows per group: one partial, ragged blocks
    T = W.laplacian_2d(2)
    run(M, M.Matrix(T), T, W.rhs(T.n, 5), act, variant=variant)


@pytest.mark.parametrize("variant", [1, 2], ids=["sr", "pipe"])
def test_refusals(M, variant):
    A = W.laplacian_2d(16)
    m = M.Matrix(A)
    for kw in ({"fallback": True}, {"precond": 1}, {"stop_rule": 1}, {"rho_fp64": 1}, {"emulate": 1},
               {"vec16": 1}, {"profile": True}, {"variant": 3}):
        with pytest.raises(M.MPCGError):
            m.set_options(**{"variant": variant, **kw})
    m.set_options(variant=variant)
    b = torch.from_numpy(W.rhs(A.n, 1)).cuda()
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    for pol in (M.Policy(kind=M.POLICY_QTABLE), M.Policy(kind=M.POLICY_FIXED, fixed_action=128)):
        m.set_policy(pol)
        with pytest.raises(M.MPCGError):
            m.solve(b, x, tol=1e-8, maxit=100)
    m.set_policy(M.Policy(kind=M.POLICY_FIXED, fixed_action=26))
    with pytest.raises(M.MPCGError):
        M.solve_batched([(m, b, x)], tol=1e-8, maxit=100)
    logging = M.Policy(kind=M.POLICY_FIXED, fixed_action=26)
    logging.rollouts_enable(64)
    m.set_policy(logging)
    with pytest.raises(M.MPCGError):
        m.solve(b, x, tol=1e-8, maxit=100)
