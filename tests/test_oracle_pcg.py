"""Pins for the oracle's preconditioned CG (section 3 with M != I: z = M^-1 r,
alpha = r^T z / p^T A p, beta = r'^T z' / r^T z, p = z + beta p; section 4.2:
M kept in fixed fp32).  M is Jacobi, diag(A).  Each pin reduces the
preconditioned solve to something fixed independently: plain CG under an exact
power-of-two similarity (bit for bit), a one-step closed form, a dense solve,
and the conjugacy and orthogonality the method guarantees.  CPU only."""
import numpy as np
import pytest

import oracle as O
import workloads as W

# actions whose dot and update formats have fp32's exponent range or more, so
# exact power-of-two scalings of the vectors commute with every rounding
WIDE = [16 * fs + 4 * fd + fa for fs in (1, 2, 3, 4) for fd in (1, 2, 3) for fa in (1, 2, 3)]


def pol(a):
    return O.OraclePolicy(fixed_action=a)


@pytest.mark.parametrize("act", [63, 42, 26, 74, 16 * 3 + 4 * 1 + 2])
def test_laplacian_pcg_equals_cg_bit_for_bit(act):
    """The 2D Laplacian's diagonal is 4 = 2^2, so M = 4I: z = r/4 exactly,
    sigma_pcg = sigma_cg / 4, p_pcg = p_cg / 4, alpha_pcg = 4 alpha_cg.  x, r and
    every residual norm are the same numbers as plain CG's, replacements
    included, as long as no replacement more than doubles the residual (which
    restarts PCG's direction only): true for these actions, whose updates are
    in fp32 or fp64 (stencil values are exact in every storage format)."""
    A = W.laplacian_2d(24)
    b = W.rhs(A.n, 3)
    kw = dict(tol=1e-8, maxit=3000, replace_period=50, fallback=True)
    x0, i0 = O.cg(A, b, policy=pol(act), **kw)
    x1, i1 = O.cg(A, b, policy=pol(act), precond=1, **kw)
    assert i0["iters"] == i1["iters"] and i0["status"] == i1["status"] == 0
    assert np.array_equal(i0["rho"], i1["rho"]) and np.array_equal(x0, x1)
    assert np.array_equal(i0["rep_rho"], i1["rep_rho"])


def scaled_pair(n, seed):
    """A1: sparse symmetric, unit diagonal, off-diagonal row sums below 1/2
    (SPD); D = diag(2^e_i); A = D A1 D has diagonal 4^e_i."""
    rng = np.random.default_rng(seed)
    A0 = W.random_spd(n, seed, spread=0.0, tmin=3, tmax=8)
    rows = np.repeat(np.arange(n), np.diff(A0.row_ptr))
    off = rows != A0.col
    v1 = np.where(off, 0.0, 1.0)
    deg = np.diff(A0.row_ptr) - 1
    # symmetric off-diagonal values: a function of the unordered pair
    lo, hi = np.minimum(rows, A0.col), np.maximum(rows, A0.col)
    h = ((lo * 7919 + hi * 104729) % 1000) / 1000.0 - 0.5
    scale = 0.45 / np.maximum(np.maximum(deg[lo], deg[hi]), 1)
    v1 = np.where(off, h * scale, v1)
    A1 = W.CSR(n, A0.row_ptr.copy(), A0.col.copy(), v1)
    e = rng.integers(-6, 7, n)
    d = 2.0 ** e
    A = W.CSR(n, A0.row_ptr.copy(), A0.col.copy(), v1 * d[rows] * d[A0.col])
    return A, A1, d


@pytest.mark.parametrize("act", [63, 42, 26, 74, 16 * 1 + 4 * 3 + 2])
def test_jacobi_pcg_is_cg_on_the_scaled_system(act):
    """With M = diag(A) = D^2, PCG on (A, b) is CG on (D^-1 A D^-1, D^-1 b) =
    (A1, D^-1 b) with x = D^-1 y, r = D r~, z = D^-1 r~, p = D^-1 p~: every
    product and sum is the scaled image of CG's, so after a fixed number of
    iterations (no replacement, which would compare norms of differently scaled
    vectors) x equals D^-1 y bit for bit."""
    A, A1, d = scaled_pair(3000, 11)
    b = W.rhs(A.n, 5)
    kw = dict(tol=1e-30, maxit=12, replace_period=0)
    x, info = O.cg(A, b, policy=pol(act), precond=1, dump=12, **kw)
    y, info1 = O.cg(A1, b / d, policy=pol(act), dump=12, **kw)
    assert info["iters"] == info1["iters"] == 12
    assert np.array_equal(x, y / d)
    assert np.array_equal(info["dump"]["r"], info1["dump"]["r"] * d)
    assert np.array_equal(info["dump"]["p"], info1["dump"]["p"] / d)
    assert np.array_equal(info["dump"]["alpha"], info1["dump"]["alpha"])


def test_jacobi_inverse_is_the_fp32_reciprocal():
    A, _, d = scaled_pair(500, 3)
    m = O.jacobi_inverse(A)
    assert m.dtype == np.float32 and np.array_equal(m.astype(np.float64), 1.0 / d ** 2)
    B = W.random_spd(400, 9, spread=2.0)
    rows = np.repeat(np.arange(B.n), np.diff(B.row_ptr))
    diag = B.val[rows == B.col]
    assert np.array_equal(O.jacobi_inverse(B), (1.0 / diag).astype(np.float32))


def test_diagonal_system_one_step():
    """A = M = diag(2^e): z = A^-1 r exactly, nu = sigma as the same sum, so
    alpha = 1 and x_1 = A^-1 b exactly; the residual is then 0."""
    n = 1000
    e = np.random.default_rng(1).integers(-10, 11, n)
    A = W.CSR(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), 2.0 ** e)
    b = W.rhs(n, 2)
    x, info = O.cg(A, b, tol=1e-12, maxit=10, precond=1, dump=2)
    assert info["status"] == 0 and info["iters"] == 1
    assert info["dump"]["alpha"][0] == 1.0
    assert np.array_equal(x, b / 2.0 ** e) and info["relres_true"] == 0.0


def test_fp64_pcg_against_dense_solve():
    for seed in (2, 3, 4):
        A = W.random_spd(60, seed, W.spread_for_kappa(1e6), tmin=2, tmax=6)
        b = W.rhs(A.n, seed)
        x, info = O.cg(A, b, tol=1e-13, maxit=200, precond=1)
        xs = np.linalg.solve(A.to_dense(), b)
        assert info["status"] == 0 and info["iters"] <= A.n
        assert np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs)


def test_preconditioned_conjugacy_and_orthogonality():
    """p_k^T A p_{k+1} = 0 and r_k^T M^-1 r_{k+1} = 0 in exact arithmetic; in
    fp64 they hold to a small multiple of the unit roundoff."""
    A = W.random_spd(2000, 7, W.spread_for_kappa(1e4))
    b = W.rhs(A.n, 7)
    x, info = O.cg(A, b, tol=1e-30, maxit=12, precond=1, dump=12)
    P, R = info["dump"]["p"], info["dump"]["r"]
    Ad = A.to_scipy() if hasattr(A, "to_scipy") else None
    m = O.jacobi_inverse(A).astype(np.float64)

    def Amul(v):
        rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
        return np.bincount(rows, weights=A.val * v[A.col], minlength=A.n)

    for k in range(11):
        ap0, ap1 = Amul(P[k]), Amul(P[k + 1])
        na = np.sqrt(P[k] @ ap0) * np.sqrt(P[k + 1] @ ap1)
        assert abs(P[k] @ ap1) <= 1e-12 * na
        nm = np.sqrt(R[k] @ (m * R[k])) * np.sqrt(R[k + 1] @ (m * R[k + 1]))
        assert abs(R[k] @ (m * R[k + 1])) <= 1e-12 * nm


def test_jacobi_removes_the_diagonal_scaling():
    """The random SPD family is D A0 D with A0 diagonally dominant and D spread
    over decades: Jacobi undoes D, so PCG needs a small fraction of CG's
    iterations, in fp64 and in every mixed action (the direction restarts at a
    replacement that more than doubles the residual)."""
    A = W.random_spd(5000, 3, W.spread_for_kappa(1e6))
    b = W.rhs(A.n, 4)
    _, i0 = O.cg(A, b, tol=1e-8, maxit=20000, policy=pol(63))
    assert i0["status"] == 0
    for act in (63, 42, 26, 74):
        _, i1 = O.cg(A, b, tol=1e-8, maxit=20000, policy=pol(act), replace_period=50, precond=1)
        assert i1["status"] == 0 and i1["relres_true"] <= 1e-8
        assert i1["iters"] * 20 < i0["iters"], (act, i1["iters"], i0["iters"])
