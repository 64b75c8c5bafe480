"""Pins for the oracle's SpMV, inner products and vector updates: exact integer
cases, rounding-error bounds against exactly rounded sums (math.fsum), exact
rational arithmetic, and hand-built cases whose result depends on the summation
order the method fixes.  CPU only."""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
import workloads as W
from test_oracle_rounding import round_fraction

U = {O.F16: 2.0 ** -11, O.BF16: 2.0 ** -8, O.F32: 2.0 ** -24, O.F64: 2.0 ** -53}
FP = {O.F16: (11, -14, 15), O.BF16: (8, -126, 127), O.F32: (24, -126, 127), O.F64: (53, -1022, 1023)}


def gamma(m, u):
    return m * u / (1 - m * u)


@pytest.mark.parametrize("fs", [O.F16, O.BF16, O.F32, O.F64])
@pytest.mark.parametrize("tier", [0, 1])
def test_spmv_laplacian_integer_exact(fs, tier):
    """Integer stencils times small integers: every intermediate is exact, so
    every format must reproduce the dense product bit for bit."""
    rng = np.random.default_rng(7)
    for A in (W.laplacian_2d(13), W.laplacian_3d(7)):
        p = rng.integers(-300, 300, A.n).astype(np.float64)
        q = O.spmv(A, p, fs, tier)
        assert np.array_equal(q, A.to_dense() @ p)


def test_spmv_fp16_row_scale():
    A = W.random_spd(400, 11, spread=2.0)
    s32, sb, sh, e = O.shadows(A)
    for i in range(A.n):
        row = A.val[A.row_ptr[i]:A.row_ptr[i + 1]]
        mx = np.max(np.abs(row))
        scaled = mx * 2.0 ** -int(e[i])
        assert 2.0 ** 14 < scaled <= 2.0 ** 15
        m, ex = math.frexp(mx)
        assert int(e[i]) == (ex - 1 if m == 0.5 else ex) - 15
    # shadows are the roundings of the fp64 values (fp16 after the exact row scale)
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    assert np.array_equal(s32, A.val.astype(np.float32).astype(np.float64))
    assert np.array_equal(sh, (A.val * 2.0 ** -e[rows].astype(np.float64)).astype(np.float16).astype(np.float64))


@pytest.mark.parametrize("fs", [O.F16, O.BF16, O.F32, O.F64])
def test_spmv_error_bound_random(fs):
    """|q_i - exact_i| within the accumulated rounding bound of the row: value
    rounding u_f, m fma roundings in acc(f), input and output conversions."""
    A = W.random_spd(300, 5, spread=1.0)
    rng = np.random.default_rng(8)
    p = rng.standard_normal(A.n).astype(np.float32).astype(np.float64)
    q = O.spmv(A, p, fs, 1)
    ua = U[O.F64] if fs == O.F64 else U[O.F32]
    for i in range(A.n):
        s, t = A.row_ptr[i], A.row_ptr[i + 1]
        prods = A.val[s:t] * p[A.col[s:t]]
        exact = float(sum(Fraction(float(a)) * Fraction(float(x))
                          for a, x in zip(A.val[s:t], p[A.col[s:t]])))
        absum = np.sum(np.abs(prods))
        m = t - s
        bound = (U[fs] + gamma(m + 1, ua)) * absum * 1.01 + 1e-300
        assert abs(q[i] - exact) <= bound


def test_spmv_csr_order_fma_chain():
    """One row [2^24, 1, -2^24] times ones: the fp32 fma chain in CSR order gives
    (2^24 + 1 -> 2^24 by ties-to-even) - 2^24 = 0; any other order gives 1."""
    n = 3
    rp = np.array([0, 3, 4, 5], np.int32)
    ci = np.array([0, 1, 2, 1, 2], np.int32)
    v = np.array([2.0 ** 24, 1.0, -(2.0 ** 24), 1.0, 1.0])
    A = W.CSR(n, rp, ci, v)
    q = O.spmv(A, np.ones(3), O.F32, 0)
    assert q[0] == 0.0
    q64 = O.spmv(A, np.ones(3), O.F64, 1)
    assert q64[0] == 1.0


@pytest.mark.parametrize("fd", [O.F16, O.BF16, O.F32, O.F64])
def test_dot_integer_exact(fd):
    rng = np.random.default_rng(9)
    for n in (0, 1, 2, 3, 5, 64, 1000, 4097):
        u = rng.integers(-8, 9, n).astype(np.float64)
        v = rng.integers(-8, 9, n).astype(np.float64)
        assert O.dot(u, v, fd) == float(int(np.dot(u.astype(np.int64), v.astype(np.int64))))


def test_dot_pairwise_structure():
    """Leaves [2^24, 1, 1, 1] in fp32: pairwise (2^24+1) + (1+1) = 2^24 + 2 (the
    first add ties to 2^24, the second is exact); the ascending chain loses
    every 1 and stays at 2^24."""
    u = np.array([2.0 ** 12, 1.0, 1.0, 1.0])
    assert O.dot(u, u, O.F32, O.ORDER_PAIRWISE) == 2.0 ** 24 + 2
    assert O.dot(u, u, O.F32, O.ORDER_SEQ) == 2.0 ** 24
    # zero padding of a non power of two length: [2^24, 1, 1] -> (2^24+1)+(1+0)
    u3 = u[:3]
    assert O.dot(u3, u3, O.F32, O.ORDER_PAIRWISE) == 2.0 ** 24


@pytest.mark.parametrize("fd", [O.F16, O.BF16, O.F32, O.F64])
def test_dot_error_bound(fd):
    rng = np.random.default_rng(10)
    for n in (7, 1000, 65537):
        u = rng.standard_normal(n)
        v = rng.standard_normal(n)
        ur = O.rd(u, fd) if fd != O.F64 else u
        vr = O.rd(v, fd) if fd != O.F64 else v
        if n <= 1000:
            exact = float(sum(Fraction(float(a)) * Fraction(float(b)) for a, b in zip(ur, vr)))
        elif fd != O.F64:
            exact = math.fsum(ur * vr)           # products of <= 24-bit values are exact
        else:
            exact = float(np.sum(np.longdouble(ur) * np.longdouble(vr)))
        ua = U[O.F64] if fd == O.F64 else U[O.F32]
        depth = math.ceil(math.log2(n)) + 1
        bound = gamma(depth, ua) * np.sum(np.abs(ur * vr)) * 1.01
        got = O.dot(u, v, fd)
        assert abs(got - exact) <= bound
        seq = O.dot(u, v, fd, O.ORDER_SEQ)
        assert abs(seq - exact) <= gamma(n + 1, ua) * np.sum(np.abs(ur * vr)) * 1.01


def test_dot_fp16_operand_overflow():
    u = np.array([7.0e4, 1.0])
    assert O.dot(u, np.ones(2), O.F16) == np.inf
    assert O.dot(u, np.ones(2), O.BF16) == 70144.0 + 1.0   # 7e4 rounds to 70144 in bf16


@pytest.mark.parametrize("fa", [O.F16, O.BF16, O.F32, O.F64])
def test_axpy_exact_rationals(fa):
    """y = rd_f(rd_acc(rd_acc(alpha) u + y)) against exact rational arithmetic."""
    rng = np.random.default_rng(11)
    n = 300
    tier_fmt = O.F64 if fa == O.F64 else O.F32
    u = O.rd(rng.standard_normal(n) * 10.0 ** rng.integers(-3, 3, n), tier_fmt)
    y = O.rd(rng.standard_normal(n), tier_fmt)
    alpha = float(rng.standard_normal() * 3)
    got = O.axpy(alpha, u, y, fa)
    acc = FP[O.F64] if fa == O.F64 else FP[O.F32]
    a_acc = round_fraction(Fraction(alpha), *acc)
    for i in range(n):
        exact = Fraction(a_acc) * Fraction(float(u[i])) + Fraction(float(y[i]))
        r1 = round_fraction(exact, *acc)
        ref = round_fraction(Fraction(r1), *FP[fa]) if math.isfinite(r1) else r1
        assert got[i] == ref
    # p update: p = rd_f(fma(beta, p, r))
    beta = 0.37
    gotp = O.xpay(beta, y, u, fa)
    b_acc = round_fraction(Fraction(beta), *acc)
    for i in range(n):
        exact = Fraction(b_acc) * Fraction(float(u[i])) + Fraction(float(y[i]))
        ref = round_fraction(Fraction(round_fraction(exact, *acc)), *FP[fa])
        assert gotp[i] == ref


def test_residual_fp64():
    A = W.laplacian_2d(9)
    rng = np.random.default_rng(12)
    x = rng.integers(-50, 50, A.n).astype(np.float64)
    b = rng.integers(-50, 50, A.n).astype(np.float64)
    assert np.array_equal(O.residual(A, b, x), b - A.to_dense() @ x)
