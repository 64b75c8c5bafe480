"""Pins for the oracle's conjugate-gradient iteration (section 3): dense
Cholesky solutions, finite termination, A-conjugacy of the directions and
orthogonality of the residuals, closed-form Laplacian spectra (directly and as
Lanczos-Ritz values from CG's alpha/beta), eigenvector right-hand sides, and the
mixed-precision reading's invariants.  CPU only."""
import math

import numpy as np
import pytest
import scipy.linalg as sla

import oracle as O
import workloads as W


def small_spd(n, seed, spread=0.5):
    return W.random_spd(n, seed, spread, tmin=2, tmax=min(8, n - 2))


@pytest.mark.parametrize("n,seed", [(16, 1), (40, 2), (64, 3)])
def test_fp64_cg_vs_cholesky(n, seed):
    A = small_spd(n, seed)
    Ad = A.to_dense()
    b = W.rhs(n, seed + 100)
    c = sla.cho_factor(Ad)
    xs = sla.cho_solve(c, b)
    kappa = np.linalg.cond(Ad)
    x, info = O.cg(A, b, tol=1e-14, maxit=10 * n)
    assert info["status"] in (0, 1)
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= max(kappa, 10) * 1e-14


def test_termination_within_n():
    """Exact arithmetic ends in at most n steps (section 3); a well-conditioned
    system reaches 1e-12 by k = n in fp64."""
    n = 24
    A = small_spd(n, 5, spread=0.0)
    assert np.linalg.cond(A.to_dense()) < 30
    b = W.rhs(n, 6)
    x, info = O.cg(A, b, tol=1e-12, maxit=n)
    assert info["status"] == 0 and info["iters"] <= n


def test_conjugacy_and_orthogonality():
    """p_i^T A p_j = 0 and r_i^T r_j = 0 for i != j (section 3), up to rounding."""
    A = W.laplacian_2d(8)
    Ad = A.to_dense()
    b = W.rhs(A.n, 3)
    kmax = 12
    x, info = O.cg(A, b, tol=1e-30, maxit=kmax, dump=kmax)
    P = info["dump"]["p"][:kmax]
    R = info["dump"]["r"][:kmax]
    G = P @ Ad @ P.T
    d = np.sqrt(np.diag(G))
    C = G / np.outer(d, d)
    off = C - np.diag(np.diag(C))
    assert np.max(np.abs(off)) < 1e-10
    Rn = R / np.linalg.norm(R, axis=1)[:, None]
    O_ = Rn @ Rn.T - np.eye(kmax)
    assert np.max(np.abs(O_)) < 1e-10


def test_laplacian_closed_form_spectrum():
    for N, d in ((6, 2), (9, 2), (4, 3), (5, 3)):
        A = W.laplacian_2d(N) if d == 2 else W.laplacian_3d(N)
        ev = np.linalg.eigvalsh(A.to_dense())
        assert np.allclose(ev, W.laplacian_eigs(N, d), rtol=0, atol=1e-12)
        assert A.nnz == W.laplacian_nnz(N, d)
    k2 = W.laplacian_eigs(64, 2)
    assert round(k2[-1] / k2[0], 2) == 1711.66
    j = np.array([1, 128])
    lam1 = 4 * np.sin(j * np.pi / 258) ** 2
    assert round(3 * lam1[1] / (3 * lam1[0]), 2) == 6743.68
    assert W.laplacian_nnz(64, 2) == 20224
    assert W.laplacian_nnz(128, 3) == 14581760


def test_lanczos_ritz_from_alpha_beta():
    """CG's alpha/beta define the Lanczos tridiagonal T_k; its extreme
    eigenvalues converge to the closed-form lambda_min and lambda_max."""
    N = 16
    A = W.laplacian_2d(N)
    b = W.rhs(A.n, 4)
    k = 120
    x, info = O.cg(A, b, tol=1e-30, maxit=k, dump=k)
    al = info["dump"]["alpha"][:k]
    be = info["dump"]["beta"][:k - 1]
    diag = 1.0 / al
    diag[1:] += be / al[:-1]
    off = np.sqrt(be) / al[:-1]
    ritz = sla.eigvalsh_tridiagonal(diag, off)
    lam = W.laplacian_eigs(N, 2)
    assert abs(ritz[-1] - lam[-1]) < 1e-8 * lam[-1]
    assert abs(ritz[0] - lam[0]) < 1e-8 * lam[-1]


def test_eigenvector_rhs_one_step():
    N = 12
    A = W.laplacian_2d(N)
    ev, V = np.linalg.eigh(A.to_dense())
    b = V[:, 5].copy()
    x, info = O.cg(A, b, tol=1e-10, maxit=10, dump=2)
    assert info["status"] == 0 and info["iters"] == 1
    assert abs(info["dump"]["alpha"][0] - 1.0 / ev[5]) < 1e-13 / ev[5]


def test_m_eigencomponents_m_steps():
    N = 12
    A = W.laplacian_2d(N)
    ev, V = np.linalg.eigh(A.to_dense())
    # distinct eigenvalues only (the 2D Laplacian has repeated ones)
    uniq = np.unique(np.round(ev, 10), return_index=True)[1]
    cols = uniq[[0, 7, 20, 33]]
    b = V[:, cols] @ np.array([1.0, -0.5, 0.25, 2.0])
    x, info = O.cg(A, b, tol=1e-11, maxit=20)
    assert info["status"] == 0 and info["iters"] == 4


def test_fp64_action_with_no_replacement_is_plain_cg():
    """Action 63 with R = 0 is textbook CG: same iterate count and residual as
    the independent native fp64 CG (different summation order, so only close)."""
    A = W.laplacian_2d(64)
    b = W.rhs(A.n, 1)
    x, info = O.cg(A, b, tol=1e-8, maxit=2000)
    x2, it2, rr2 = O.cg_plain(A, b, tol=1e-8, maxit=2000)
    assert info["status"] == 0
    assert abs(info["iters"] - it2) <= 1
    xs = np.linalg.solve(A.to_dense(), b)
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1712 * 1e-8


def test_laplacian_spmv_format_invariance_of_history():
    """Integer stencils are exact in every format, so actions that differ only in
    the SpMV format give bit-identical histories."""
    A = W.laplacian_3d(12)
    b = W.rhs(A.n, 2)
    outs = []
    for fs in range(3):
        pol = O.OraclePolicy(fixed_action=16 * fs + 4 * 2 + 2)
        x, info = O.cg(A, b, tol=1e-8, maxit=2000, policy=pol, replace_period=50)
        outs.append((x, info["rho"]))
    for x, rho in outs[1:]:
        assert np.array_equal(x, outs[0][0]) and np.array_equal(rho, outs[0][1])


@pytest.mark.parametrize("action", [0 * 16 + 2 * 4 + 2, 1 * 16 + 2 * 4 + 2])
def test_mixed_fixed_reaches_tolerance(action):
    A = W.laplacian_3d(20)
    b = W.rhs(A.n, 2)
    pol = O.OraclePolicy(fixed_action=action)
    x, info = O.cg(A, b, tol=1e-8, maxit=3000, policy=pol, replace_period=50)
    assert info["status"] == 0 and info["relres_true"] <= 1e-8
    r = b - A.to_dense() @ x if A.n < 3000 else O.residual(A, b, x)
    assert np.linalg.norm(r) / np.linalg.norm(b) <= 1e-8
    x64, i64 = O.cg(A, b, tol=1e-8, maxit=3000)
    assert info["iters"] <= 1.25 * i64["iters"]
    # the recursive residual tracks the true one between replacements
    assert np.all(np.abs(np.log10(info["rep_rho"]) - np.log10(info["rho"][info["rep_k"]])) < 3)


def test_pairwise_and_sequential_orders_agree_on_iterations():
    A = W.random_spd(3000, 21, spread=1.0)
    b = W.rhs(A.n, 22)
    pol = O.OraclePolicy(fixed_action=1 * 16 + 2 * 4 + 2)
    _, a = O.cg(A, b, tol=1e-8, maxit=20000, policy=pol, replace_period=50)
    _, s = O.cg(A, b, tol=1e-8, maxit=20000, policy=pol, replace_period=50, order=O.ORDER_SEQ)
    assert a["status"] == 0 and s["status"] == 0
    assert abs(a["iters"] - s["iters"]) <= 0.05 * s["iters"]


def test_status_edge_cases():
    A = W.laplacian_2d(10)
    b = W.rhs(A.n, 1)
    x, info = O.cg(A, b, maxit=0)
    assert info["status"] == 1 and info["iters"] == 0
    x, info = O.cg(A, np.zeros(A.n), maxit=10)
    assert info["status"] == 0 and np.all(x == 0)
    bn = b.copy()
    bn[3] = np.nan
    x, info = O.cg(A, bn, maxit=10)
    assert info["status"] == 3
    # x0 that already solves the system
    xs = np.linalg.solve(A.to_dense(), b)
    x, info = O.cg(A, b, x0=xs, tol=1e-8, maxit=10)
    assert info["status"] == 0 and info["iters"] == 0


def test_indefinite_breaks_down():
    A = W.laplacian_2d(10)
    A.val = A.val.copy()
    diag = A.col == np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    A.val[diag] = -4.0
    b = W.rhs(A.n, 1)
    x, info = O.cg(A, b, maxit=50)
    # -L is negative definite: nu < 0 at the first step
    assert info["status"] == 3 and info["iters"] == 0
    x, info = O.cg(A, b, maxit=50, fallback=True)
    assert info["status"] == 3


def test_fp16_hostile_falls_back_and_converges():
    """D-scaled entries far above 65504: the all-fp16 action overflows (dot of
    fp16 operands) or stagnates; the fp64 fallback then converges (status 2)."""
    A = W.random_spd(2000, 31, spread=3.0)
    b = W.rhs(A.n, 32) * 1e6
    pol = O.OraclePolicy(fixed_action=0)
    x, info = O.cg(A, b, tol=1e-8, maxit=20000, policy=pol, replace_period=50, fallback=True)
    assert info["fallback_at"] >= 0
    assert info["status"] == 2 and info["relres_true"] <= 1e-8
    assert np.all(info["actions"][info["fallback_at"]:] == 63)
    x2, info2 = O.cg(A, b, tol=1e-8, maxit=20000, policy=pol, replace_period=50, fallback=False)
    assert info2["status"] in (1, 3)
