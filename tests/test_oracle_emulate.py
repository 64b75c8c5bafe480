"""The paper's emulation reading in the oracle (emulate = 1), pinned by hand.

Section 4 writes fl_p(op) for an operation computed in precision p, and the
paper emulates the formats in software.  Read as "compute in fp64, round the
operation's result to p", with every vector in fp64: the SpMV rounds each
q_i of the fp64 row sum (no row scale), a dot rounds its fp64 total, an update
rounds each fp64 fma.  The expected values below are worked out with exact
rational arithmetic (Fraction) and a rounding written from the format
definition, independently of the oracle's code."""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
import workloads as W


def rd_bits(v: float, t: int) -> float:
    """Round a normal double to t significant bits, ties to even (Python's
    round() on an exactly representable double is round-half-even)."""
    if v == 0.0:
        return v
    m, e = math.frexp(v)
    return math.ldexp(round(math.ldexp(m, t)), e - t)


def fma_exact(a: float, b: float, c: float) -> float:
    return float(Fraction(a) * Fraction(b) + Fraction(c))   # one rounding


def one_by_one(a, b=1.0):
    return W.CSR(1, np.array([0, 1], np.int32), np.array([0], np.int32), np.array([a]))


def test_fp64_action_is_the_hardware_reading():
    A = W.laplacian_2d(14)
    b = W.rhs(A.n, 2)
    for kw in ({}, {"precond": 1}, {"rho_fp64": 1}):
        x1, i1 = O.cg(A, b, tol=1e-10, maxit=500, replace_period=50, emulate=1, **kw)
        x0, i0 = O.cg(A, b, tol=1e-10, maxit=500, replace_period=50, **kw)
        k = i0["iters"]
        assert i1["iters"] == k and np.array_equal(i1["rho"][:k + 1], i0["rho"][:k + 1]) and np.array_equal(x1, x0)


def test_update_rounding_by_hand():
    """A = [3], b = [1], action (fp64, fp64, bf16): alpha = fl(1/3); the
    update rounds fma(-alpha, 3, 1) = 1 - 3 fl(1/3) = 2^-54 exactly to bf16
    (exact), so rho_1 = 2^-54 and x = rd_bf16(fl(1/3)).  The hardware reading
    rounds alpha to fp32 first and its residual is about 3e-8."""
    a = 16 * 3 + 4 * 3 + 1
    pol = O.OraclePolicy(fixed_action=a)
    alpha = 1.0 / 3.0
    r1 = rd_bits(fma_exact(-alpha, 3.0, 1.0), 8)
    assert r1 == 2.0 ** -54
    x, info = O.cg(one_by_one(3.0), np.array([1.0]), tol=1e-300, maxit=1, policy=pol, replace_period=50, emulate=1)
    assert info["rho"][1] == r1 and x[0] == rd_bits(alpha, 8)
    _, info_hw = O.cg(one_by_one(3.0), np.array([1.0]), tol=1e-300, maxit=1, policy=pol, replace_period=50)
    assert abs(info_hw["rho"][1] - 2.98e-8) < 1e-9


def test_dot_rounding_by_hand():
    """A = [3 + 2^-8], b = [1], action (fp64, bf16, fp64): nu = rd_bf16(3 + 2^-8)
    = 3 (a quarter unit above 3), alpha = fl(1/3), r_1 = fma(-alpha, 3 + 2^-8, 1)
    in fp64, sigma' = rd_bf16(r_1^2) and rho_1 = sqrt(sigma')."""
    a = 16 * 3 + 4 * 1 + 3
    q = 3.0 + 2.0 ** -8
    assert rd_bits(q, 8) == 3.0
    alpha = 1.0 / 3.0
    r1 = fma_exact(-alpha, q, 1.0)
    rho1 = math.sqrt(rd_bits(r1 * r1, 8))
    _, info = O.cg(one_by_one(q), np.array([1.0]), tol=1e-300, maxit=1, policy=O.OraclePolicy(fixed_action=a),
                   replace_period=50, emulate=1, dump=2)
    assert info["dump"]["alpha"][0] == alpha
    assert info["rho"][1] == rho1


def test_spmv_result_rounding_on_integers():
    """Integer 2D Laplacian and integer b: every fp64 sum is exact, so the
    first SpMV is rd_bf16(A b) elementwise and alpha_0 = (b.b) / (b.rd_bf16(A b)).
    The hardware reading stores A in bf16 (exact here) and rounds nothing."""
    A = W.laplacian_2d(16)
    rng = np.random.default_rng(7)
    b = rng.integers(-200, 201, A.n).astype(np.float64)
    q = A.to_dense() @ b
    qb = np.array([rd_bits(v, 8) for v in q])
    assert not np.array_equal(qb, q)
    a = 16 * 1 + 4 * 3 + 3
    _, info = O.cg(A, b, tol=1e-300, maxit=1, policy=O.OraclePolicy(fixed_action=a), replace_period=50,
                   emulate=1, dump=2)
    assert info["dump"]["alpha"][0] == float(b @ b) / float(b @ qb)
    _, hw = O.cg(A, b, tol=1e-300, maxit=1, policy=O.OraclePolicy(fixed_action=a), replace_period=50, dump=2)
    assert hw["dump"]["alpha"][0] == float(b @ b) / float(b @ q)


@pytest.mark.parametrize("emulate,status", [(1, 3), (0, 0)])
def test_fp16_result_overflow_without_row_scale(emulate, status):
    """A = [1e5]: the emulated fp16 SpMV rounds q = 1e5 to infinity (no row
    scale) and breaks down; the hardware reading scales the row and converges."""
    a = 16 * 0 + 4 * 3 + 3
    _, info = O.cg(one_by_one(1e5), np.array([1.0]), tol=1e-8, maxit=20, policy=O.OraclePolicy(fixed_action=a),
                   replace_period=50, emulate=emulate)
    assert info["status"] == status
