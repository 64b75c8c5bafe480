"""Structure of the seeded synthetic inputs (sizes, symmetry, SPD, nnz/row ranges). CPU only."""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

import workloads as W


def to_scipy(A):
    return sp.csr_matrix((A.val, A.col, A.row_ptr), shape=(A.n, A.n))


def test_laplacian_sizes():
    A = W.laplacian_2d(64)
    assert A.n == 4096 and A.nnz == 20224
    assert A.row_lengths().max() == 5 and A.row_lengths().min() == 3
    S = to_scipy(W.laplacian_3d(10))
    assert abs(S - S.T).max() == 0


def test_random_spd_structure():
    A = W.random_spd(20000, 3, spread=1.5)
    L = A.row_lengths()
    assert L.min() >= 2 and L.max() <= 27 and 15 <= L.mean() <= 19
    assert np.mean(L >= 9) > 0.99
    S = to_scipy(A)
    assert abs(S - S.T).max() == 0
    assert np.all(np.diff(A.col[A.row_ptr[5]:A.row_ptr[6]]) > 0)
    B = W.random_spd(300, 4, spread=2.0)
    sla.cholesky(B.to_dense())                     # SPD
    assert np.array_equal(W.random_spd(300, 4, 2.0).val, B.val)   # seeded


def test_banded_structure():
    A = W.banded_spd(500, 7, 9, spread=1.0)
    L = A.row_lengths()
    assert L.max() == 15 and L.min() == 8
    sla.cholesky(A.to_dense())


def test_rhs_and_families():
    b = W.rhs(1000, 1)
    assert b.min() >= -1 and b.max() <= 1
    for s in (300, 301, 302):
        A = W.family_system(s, n_lo=1e3, n_hi=5e3)
        assert 500 <= A.n <= 6000
    A = W.batch_system(1001, n_hi=3e3)
    assert A.row_lengths().max() <= 27


def test_bbt_system_is_the_dense_product():
    """A = B B^T + beta I rebuilt densely from the same draws (section 5.1)."""
    for reading in ("pairs", "percent"):
        n = 300
        A = W.bbt_system(4, n=n, density_reading=reading)
        rng = np.random.default_rng(4)
        m = n if reading == "pairs" else int(round(0.01 * n * n))
        bi, bj, bv = rng.integers(0, n, m), rng.integers(0, n, m), rng.standard_normal(m)
        beta = rng.uniform(1e-4, 1e-2)
        B = np.zeros((n, n))
        np.add.at(B, (bi, bj), bv)
        want = B @ B.T + beta * np.eye(n)
        D = A.to_dense()
        assert np.array_equal(D, D.T)
        assert np.allclose(D, want, rtol=1e-12, atol=1e-12)
        assert 1e-4 <= beta <= 1e-2
        np.linalg.cholesky(D)


def test_poisson_subdomain_structure():
    """5-point stencil with spacings hx, hy of the random subdomain: A is
    cx (I x T) + cy (T x I), T = tridiag(-1, 2, -1); away from the boundary b is
    the source term alone."""
    for seed in range(6):
        A, b = W.poisson_subdomain(seed, N=12)
        D = A.to_dense()
        N = 12
        T = 2 * np.eye(N) - np.eye(N, k=1) - np.eye(N, k=-1)
        cx = -D[0, 1]
        cy = -D[0, N]
        assert cx > 0 and cy > 0
        assert np.allclose(D, cx * np.kron(np.eye(N), T) + cy * np.kron(T, np.eye(N)), rtol=1e-14)
        np.linalg.cholesky(D)
        assert b.shape == (N * N,) and np.all(np.isfinite(b))
