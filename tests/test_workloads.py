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
