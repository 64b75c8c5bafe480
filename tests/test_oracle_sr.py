"""The oracle's single-reduction CG (Chronopoulos-Gear) and pipelined CG
(Ghysels-Vanroose), pinned by hand and by the mathematics.

The single-reduction variant rearranges section 3's CG so that an iteration
takes both inner products (gamma = r.r, delta = r.w with w = A r) right after
its one SpMV and carries s = A p by a recurrence; the pipelined one carries
w = A r and z = A s by recurrences too, so its SpMV q = A w does not wait for
the inner products.  In exact arithmetic both give section 3's iterates, so
the same hand-worked values pin both.  The pins:
  * a 2x2 system whose two iterations are worked out by hand (alpha, beta, the
    recurrence s, the solution, the recursive residual);
  * one bf16 and one fp32 update on 3I, whose rounded values are fixed by hand
    (and where the recursive and the true residual differ);
  * in fp64, the iterates of section 3's CG and the dense solution, finite
    termination on a matrix with m distinct eigenvalues, conjugate directions
    and orthogonal residuals, and s = A p;
  * the replacement: s recomputed as A p after each one, the history, the
    flags, and the true relres of the returned x;
  * the degenerate cases: b = 0, an exact initial guess, maxit = 0, an
    indefinite matrix (breakdown at the first step), actions outside the set;
  * for the pipelined variant, w = A r and z = A s on the hand-worked 2x2 and
    in fp64, and their recomputation at each replacement."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
import workloads as W

VARIANTS = {"sr": O.cg_sr, "pipe": O.cg_pipe}


def csr(dense):
    d = np.asarray(dense, dtype=np.float64)
    rows, cols = np.nonzero(d)
    return W._from_coo(d.shape[0], rows, cols, d[rows, cols], "dense")


def spm(A):
    return sp.csr_matrix((A.val, A.col, A.row_ptr), shape=(A.n, A.n))


@pytest.mark.parametrize("var", ["sr", "pipe"])
def test_two_by_two_by_hand(var):
    """A = diag(2, 1), b = (1, 1).  By hand: w0 = (2, 1), gamma0 = 2,
    delta0 = 3, alpha0 = 2/3; r1 = (-1/3, 1/3), w1 = (-2/3, 1/3),
    gamma1 = 2/9, delta1 = 1/3, beta1 = 1/9,
    alpha1 = (2/9) / (1/3 - (1/9)(2/9)(3/2)) = 3/4; p1 = (-2/9, 4/9),
    s1 = w1 + beta1 s0 = (-4/9, 4/9) = A p1; x2 = (1/2, 1), r2 = 0."""
    A = csr([[2.0, 0.0], [0.0, 1.0]])
    x, info = VARIANTS[var](A, [1.0, 1.0], 63, tol=1e-12, maxit=10, dump=2)
    d = info["dump"]
    if var == "pipe":
        # w0 = A r0 = (2, 1), w1 = w0 - alpha0 z0 = (-2/3, 1/3) = A r1;
        # z0 = q0 = A w0 = (4, 1), z1 = A w1 + beta1 z0 = (-8/9, 4/9) = A s1
        np.testing.assert_allclose(d["w"][0], [2.0, 1.0], rtol=0)
        np.testing.assert_allclose(d["w"][1], [-2 / 3, 1 / 3], rtol=1e-15)
        np.testing.assert_allclose(d["z"][0], [4.0, 1.0], rtol=0)
        np.testing.assert_allclose(d["z"][1], [-8 / 9, 4 / 9], rtol=1e-15)
    assert info["status"] == 0 and info["iters"] == 2
    np.testing.assert_allclose(d["alpha"], [2 / 3, 3 / 4], rtol=1e-15)
    np.testing.assert_allclose(d["beta"], [0.0, 1 / 9], rtol=1e-15)
    np.testing.assert_allclose(d["p"][1], [-2 / 9, 4 / 9], rtol=1e-15)
    np.testing.assert_allclose(d["s"][0], [2.0, 1.0], rtol=0)
    np.testing.assert_allclose(d["s"][1], [-4 / 9, 4 / 9], rtol=1e-15)
    np.testing.assert_allclose(d["r"][1], [-1 / 3, 1 / 3], rtol=1e-15)
    np.testing.assert_allclose(x, [0.5, 1.0], rtol=1e-15)
    assert info["rho"][0] == 1.0
    assert info["rho"][1] == pytest.approx(1 / 3, rel=1e-15)   # sqrt(2/9) / sqrt(2)
    assert list(info["rep_k"]) == [2]                            # rho_2 = 0 triggers the check
    assert info["flags"][1] == O.FL_REPLACED and info["flags"][0] == 0
    assert list(info["actions"]) == [63, 63]


@pytest.mark.parametrize("var", ["sr", "pipe"])
@pytest.mark.parametrize("fa,x_exp", [(O.BF16, 0.333984375), (O.F32, 11184811 * 2.0**-25)])
def test_one_low_precision_update_by_hand(fa, x_exp, var):
    """A = 3I (2x2), b = (1, 1): alpha0 = 1/3 (fp64), x_lo = rd_fa(fp32(1/3)):
    bf16 keeps 8 significant bits, 1.0101011b x 2^-2 = 0.333984375; fp32 gives
    11184811 x 2^-25.  r1 = rd_fa(1 - 3 fp32(1/3)) = -2^-25 in both (exact), so
    the recursive rho_1 = 2^-25, while the true relres of x is |1 - 3 x|:
    2^-9 with bf16 updates, 2^-25 with fp32 ones."""
    A = csr([[3.0, 0.0], [0.0, 3.0]])
    act = O.action(O.BF16, O.F32, fa)
    x, info = VARIANTS[var](A, [1.0, 1.0], act, tol=1e-12, maxit=1, dump=1)
    assert info["status"] == 1 and info["iters"] == 1
    assert info["dump"]["alpha"][0] == 1 / 3
    assert list(x) == [x_exp, x_exp]
    assert info["rho"][1] == pytest.approx(2.0**-25, rel=1e-15)
    assert info["relres_true"] == pytest.approx(abs(1 - 3 * x_exp), rel=1e-15)
    assert info["relres_true"] == pytest.approx(2.0**-9 if fa == O.BF16 else 2.0**-25, rel=1e-15)


@pytest.mark.parametrize("var", ["sr", "pipe"])
@pytest.mark.parametrize("A_fn", [lambda: W.laplacian_2d(24), lambda: W.random_spd(400, 3, 1.0)],
                         ids=["lap2d_24", "rspd_400"])
def test_fp64_iterates_are_those_of_cg(A_fn, var):
    """In fp64 the single-reduction iterates are section 3's: the same
    iteration count as the oracle's CG (the pipelined ones within 5 %), the
    same x to rounding, the dense solution, and the recurrences s = A p (and
    w = A r, z = A s) to rounding."""
    A = A_fn()
    b = W.rhs(A.n, 4)
    x, info = VARIANTS[var](A, b, 63, tol=1e-10, maxit=2000, dump=40)
    x2, info2 = O.cg(A, b, tol=1e-10, maxit=2000, policy=O.OraclePolicy(fixed_action=63))
    assert info["status"] == 0 and info2["status"] == 0
    if var == "sr":
        assert info["iters"] == info2["iters"]
    else:
        # pipelining propagates the rounding errors of its recurrences further
        # (Cools et al.): in fp64 a few more iterations on the random SPD
        assert abs(info["iters"] - info2["iters"]) <= 0.05 * info2["iters"]
    assert np.abs(x - x2).max() <= 1e-9 * np.abs(x2).max()
    xd = np.linalg.solve(A.to_dense(), b)
    assert np.abs(x - xd).max() <= 1e-7 * np.abs(xd).max()
    S = spm(A)
    m = min(40, info["iters"])
    P = info["dump"]["p"][:m]
    AP = (S @ P.T).T
    for k in range(m):
        np.testing.assert_allclose(info["dump"]["s"][k], AP[k], atol=1e-10 * np.abs(AP[k]).max())
    if var == "pipe":
        AR = (S @ info["dump"]["r"][:m].T).T
        AS = (S @ info["dump"]["s"][:m].T).T
        for k in range(m):
            np.testing.assert_allclose(info["dump"]["w"][k], AR[k], atol=1e-10 * np.abs(AR[k]).max())
            np.testing.assert_allclose(info["dump"]["z"][k], AS[k], atol=1e-10 * np.abs(AS[k]).max())
    # A-conjugate directions, orthogonal residuals (relative to their norms)
    G = P @ AP.T
    dg = np.sqrt(np.diag(G))
    C = np.abs(G) / np.outer(dg, dg)
    Rm = info["dump"]["r"][:m]
    Gr = np.abs(Rm @ Rm.T) / np.outer(np.linalg.norm(Rm, axis=1), np.linalg.norm(Rm, axis=1))
    off = ~np.eye(m, dtype=bool)
    near = np.abs(np.subtract.outer(np.arange(m), np.arange(m))) <= 3
    assert C[off & near].max() < 1e-8 and Gr[off & near].max() < 1e-8


@pytest.mark.parametrize("var", ["sr", "pipe"])
def test_finite_termination_on_distinct_eigenvalues(var):
    """A diagonal matrix with 5 distinct eigenvalues and b touching all of
    them: the Krylov space has dimension 5, so CG ends after 5 iterations."""
    ev = np.repeat([1.0, 2.0, 3.0, 5.0, 8.0], 12)
    A = csr(np.diag(ev))
    b = np.linspace(0.5, 1.5, ev.size)
    x, info = VARIANTS[var](A, b, 63, tol=1e-12, maxit=50)
    assert info["status"] == 0 and info["iters"] == 5
    np.testing.assert_allclose(x, b / ev, rtol=1e-13)


def test_replacement_recomputes_s():
    """bf16 updates, replacement every 5 iterations.  Between replacements the
    recurrence s drifts from A p by bf16 roundings, and the gap
    ||s_k - A p_k|| / ||A p_k|| (in fp64, from the dumped p and s) grows; the
    first update after a replacement takes s' = A p recomputed, so there the
    gap falls back to about its size after one step (here by 30-55 %, while
    steps without a replacement change it by under 10 %)."""
    A = W.laplacian_2d(80)
    b = W.rhs(A.n, 6)
    R = 5
    act = O.action(O.F32, O.F32, O.BF16)
    x, info = O.cg_sr(A, b, act, tol=1e-8, maxit=40, replace_period=R, dump=40)
    assert info["iters"] == 40
    S = spm(A)
    P, Sv = info["dump"]["p"], info["dump"]["s"]
    AP = (S @ P.T).T
    gap = np.linalg.norm(Sv - AP, axis=1) / np.linalg.norm(AP, axis=1)
    sync = list(range(R, 40, R))
    assert list(info["rep_k"]) == sync + [40]
    for k in sync:
        assert gap[k] < 0.75 * gap[k - 1], (k, gap[k - 1], gap[k])
    rest = [k for k in range(2, 40) if k % R]
    assert all(gap[k] > 0.9 * gap[k - 1] for k in rest)


def test_history_flags_and_true_relres():
    A = W.laplacian_2d(50)
    b = W.rhs(A.n, 7)
    R = 7
    x, info = O.cg_sr(A, b, O.action(O.BF16, O.F32, O.F32), tol=1e-8, maxit=2000, replace_period=R)
    assert info["status"] == 0
    k = info["iters"]
    rep = list(info["rep_k"])
    assert rep[:-1] == list(range(R, k, R))[:len(rep) - 1]
    assert rep[-1] == k
    for j, rk in enumerate(rep):
        assert info["rho"][rk] == info["rep_rho"][j]
        assert info["flags"][rk - 1] & O.FL_REPLACED
    assert np.count_nonzero(info["flags"] & O.FL_REPLACED) == len(rep)
    tr = np.linalg.norm(b - spm(A) @ x) / np.linalg.norm(b)
    assert info["relres_true"] == pytest.approx(tr, rel=1e-5)
    assert info["relres_true"] <= 1e-8
    # the recursive residual before the last check is <= tol unless k is a multiple of R
    if k % R:
        assert info["rho"][k] <= 1e-8


@pytest.mark.parametrize("var", ["sr", "pipe"])
def test_degenerate_cases(var):
    cg = VARIANTS[var]
    A = W.laplacian_2d(6)
    x, info = cg(A, np.zeros(A.n), 26)
    assert info["status"] == 0 and info["iters"] == 0 and info["rho"][0] == 0.0 and not x.any()
    xs = np.linalg.solve(A.to_dense(), W.rhs(A.n, 1))
    b = A.to_dense() @ xs
    x, info = cg(A, b, 26, x0=xs, tol=1e-8)
    assert info["status"] == 0 and info["iters"] == 0
    x, info = cg(A, W.rhs(A.n, 1), 26, maxit=0)
    assert info["status"] == 1 and info["iters"] == 0 and info["rho"][0] == 1.0
    # diag(1, -1), b = (1, 1): delta0 = r.A r = 0, no positive step
    x, info = cg(csr([[1.0, 0.0], [0.0, -1.0]]), [1.0, 1.0], 63)
    assert info["status"] == 3 and info["iters"] == 0
    assert info["relres_true"] == 1.0
    for bad in (80, 128, -1):
        with pytest.raises(ValueError):
            cg(A, W.rhs(A.n, 1), bad)


def test_pipelined_replacement_recomputes_w_and_z():
    """fp32 actions, replacement every 5 iterations: w (the recurrence for
    A r) is rd(A r) again at each replacement, so its gap ||w - A r|| / ||A r||
    is one fp32 rounding there (under 1 u) and grows between replacements
    (over 5 u four steps later); z (for A s) is recomputed from the new s, and
    its gap falls at each replacement."""
    A = W.laplacian_2d(80)
    b = W.rhs(A.n, 6)
    R = 5
    x, info = O.cg_pipe(A, b, O.action(O.F32, O.F32, O.F32), tol=1e-8, maxit=40, replace_period=R, dump=40)
    assert info["iters"] == 40 and list(info["rep_k"]) == list(range(R, 41, R))
    S = spm(A)
    d = info["dump"]
    AR = (S @ d["r"].T).T
    AS = (S @ d["s"].T).T
    gw = np.linalg.norm(d["w"] - AR, axis=1) / np.linalg.norm(AR, axis=1)
    gz = np.linalg.norm(d["z"] - AS, axis=1) / np.linalg.norm(AS, axis=1)
    u = 2.0**-24
    for k in range(0, 40, R):
        assert gw[k] < 1.0 * u
        assert gw[k + R - 1] > 5.0 * u
    for k in range(R, 40, R):
        assert gz[k] < 0.75 * gz[k - 1]
