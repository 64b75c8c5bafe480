"""16-bit vector storage in the oracle (vec16), pinned.

With bf16 updates every update already rounds r, p and x_lo to bf16, so
holding them in bf16 containers changes nothing there; what changes is a
start, replacement or tier switch, where r and p are rounded to bf16 instead
of fp32.  Pinned: actions without bf16 updates are unaffected, every r and p
an iteration sees is bf16-representable, and one iteration worked by hand."""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W


def rd_bits(v: float, t: int) -> float:
    if v == 0.0:
        return v
    m, e = math.frexp(v)
    return math.ldexp(round(math.ldexp(m, t)), e - t)


@pytest.mark.parametrize("act", [63, 16 * 1 + 4 * 2 + 2, 0, 16 * 2 + 4 * 1 + 0])
def test_other_update_formats_are_unaffected(act):
    A = W.laplacian_2d(20)
    b = W.rhs(A.n, 3)
    pol = O.OraclePolicy(fixed_action=act)
    x1, i1 = O.cg(A, b, tol=1e-8, maxit=600, policy=pol, replace_period=50, fallback=True, vec16=1)
    x0, i0 = O.cg(A, b, tol=1e-8, maxit=600, policy=pol, replace_period=50, fallback=True)
    k = i0["iters"]
    assert i1["iters"] == k and np.array_equal(i1["rho"][:k + 1], i0["rho"][:k + 1]) and np.array_equal(x1, x0)


def test_vectors_are_bf16_at_every_iteration():
    """Action (fp32 SpMV, fp32 dot, bf16 update) with replacements every 10
    iterations: every dumped p and r is bf16-representable with vec16; without
    it p_0 and the replaced r carry fp32 values."""
    A = W.laplacian_2d(12)
    b = W.rhs(A.n, 4)
    act = 16 * 2 + 4 * 2 + 1
    pol = O.OraclePolicy(fixed_action=act)
    _, info = O.cg(A, b, tol=1e-12, maxit=40, policy=pol, replace_period=10, vec16=1, dump=40)
    k = info["iters"]
    for name in ("p", "r"):
        v = info["dump"][name][:k]
        assert np.array_equal(O.rd(v.ravel(), O.BF16), v.ravel()), name
    _, base = O.cg(A, b, tol=1e-12, maxit=40, policy=pol, replace_period=10, dump=40)
    p0 = base["dump"]["p"][0]
    assert not np.array_equal(O.rd(p0, O.BF16), p0)


def test_one_iteration_by_hand():
    """A = [2], b = [1 + 2^-10], action (fp32, fp32, bf16): with vec16 the
    start rounds r_0 = p_0 = rd_bf16(b) = 1, so q = 2, nu = 2 (fp32),
    alpha = sigma / nu with sigma = b^2 in fp64, and the update gives
    r_1 = rd_bf16(fma_fp32(-fl32(alpha), 2, 1)); rho_1 = sqrt(fl32(r_1^2)) / b."""
    b0 = 1.0 + 2.0 ** -10
    A = W.CSR(1, np.array([0, 1], np.int32), np.array([0], np.int32), np.array([2.0]))
    act = 16 * 2 + 4 * 2 + 1
    pol = O.OraclePolicy(fixed_action=act)
    _, info = O.cg(A, np.array([b0]), tol=1e-300, maxit=1, policy=pol, replace_period=50, vec16=1)
    assert rd_bits(b0, 8) == 1.0
    alpha = (b0 * b0) / 2.0
    a32 = float(np.float32(alpha))
    r1 = rd_bits(1.0 - 2.0 * a32, 8)        # exact in fp32 (Sterbenz), then bf16
    rho1 = math.sqrt(float(np.float32(r1) * np.float32(r1))) / b0
    assert info["rho"][1] == rho1
    _, base = O.cg(A, np.array([b0]), tol=1e-300, maxit=1, policy=pol, replace_period=50)
    assert base["rho"][1] != rho1
