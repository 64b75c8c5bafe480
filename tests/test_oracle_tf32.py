"""tf32 in the oracle, pinned to what fixes it independently of its code.

tf32 (section 5's format set; not in Table 1) is fp32's exponent range with an
11-bit significand, the same significand as fp16.  So on fp16's normal range
it rounds exactly like fp16 (numpy's float16 conversion, an independent
implementation); elsewhere a power-of-two scale moves any value into that
range without changing the rounding.  The SpMV, dot and axpy at tf32 then
follow from the rounding: pinned against fp32 operations on pre-rounded
operands, and against fp16 where the two formats coincide.  The action
encoding and the per-operation tables over five formats are pinned by hand."""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W


def tf32_via_fp16(x):
    """Round to tf32 through numpy's float16: scale |x| into [1, 2); in the top
    binades scale by 2^-112 and in tf32's subnormal range by 2^112, which maps
    fp16's own overflow threshold and subnormal grid onto tf32's; round, scale
    back."""
    out = np.empty_like(x)
    for i, v in enumerate(x):
        if v == 0.0 or not math.isfinite(v):
            out[i] = v
            continue
        e = math.frexp(abs(v))[1] - 1
        s = 112 if e >= 98 else (-112 if e < -126 else e)
        with np.errstate(over="ignore"):          # fp16 overflow is the point at the top
            out[i] = math.ldexp(float(np.float16(math.ldexp(v, -s))), s)
    return out


def test_rounding_matches_fp16_route_over_the_whole_range():
    rng = np.random.default_rng(1)
    x = rng.standard_normal(20000) * np.exp2(rng.uniform(-149, 128, 20000))
    x = np.concatenate([x, rng.standard_normal(2000) * np.exp2(rng.uniform(-140, -120, 2000))])
    got = O.rd(x, O.TF32)
    want = tf32_via_fp16(x)
    assert np.array_equal(got, want)


def test_rounding_special_values():
    u = 2.0 ** -11
    cases = {
        1 + u: 1.0,                                   # tie, even stays
        1 + 3 * u: 1 + 2 ** -9,                       # tie, rounds to the even neighbour
        (2 - 2 ** -10) * 2.0 ** 127: (2 - 2 ** -10) * 2.0 ** 127,   # largest finite
        (2 - 2 ** -11) * 2.0 ** 127: math.inf,        # the midpoint to 2^128 overflows
        2.0 ** -136: 2.0 ** -136,                     # smallest subnormal
        2.0 ** -137: 0.0,                             # half of it: tie to even zero
        1.5 * 2.0 ** -137: 2.0 ** -136,
        69632.0: 69632.0,                             # 2^16 + 2^12: beyond fp16, exact in tf32
        70000.0: 70016.0,                             # 11 significant bits: steps of 64 here
        1e-40: round(1e-40 / 2.0 ** -136) * 2.0 ** -136,
    }
    for x, want in cases.items():
        assert O.rd(np.array([x]), O.TF32)[0] == want, x
        assert O.rd(np.array([-x]), O.TF32)[0] == -want, x


def _csr_with(A, vals):
    return W.CSR(A.n, A.row_ptr, A.col, np.asarray(vals, dtype=np.float64))


@pytest.mark.parametrize("tier", [0, 1])
def test_spmv_is_fp32_spmv_of_the_rounded_matrix(tier):
    A = W.random_spd(3000, 2, spread=15.0)          # entries over many binades, inside fp32
    rng = np.random.default_rng(3)
    p = rng.standard_normal(A.n)
    p = p.astype(np.float32).astype(np.float64) if tier == 0 else p
    At = _csr_with(A, tf32_via_fp16(A.val))
    assert np.array_equal(O.shadow_tf32(A), At.val)
    assert np.array_equal(O.spmv(A, p, O.TF32, tier), O.spmv(At, p, O.F32, tier))
    # an integer stencil is exact in both formats
    L = W.laplacian_3d(12)
    p2 = rng.standard_normal(L.n).astype(np.float32).astype(np.float64)
    assert np.array_equal(O.spmv(L, p2, O.TF32, 0), O.spmv(L, p2, O.F32, 0))


def test_dot_and_axpy_coincide_with_fp16_on_its_normal_range():
    rng = np.random.default_rng(4)
    n = 4099
    u = rng.uniform(0.5, 2.0, n) * rng.choice([-1, 1], n) * 2.0 ** rng.integers(-6, 6, n)
    v = rng.uniform(0.5, 2.0, n) * 2.0 ** rng.integers(-6, 6, n)
    assert O.dot(u, v, O.TF32) == O.dot(u, v, O.F16)
    y = rng.uniform(0.5, 2.0, n) * 2.0 ** rng.integers(-3, 3, n)
    alpha = 0.3125
    assert np.array_equal(O.axpy(alpha, u, y, O.TF32), O.axpy(alpha, u, y, O.F16))
    # beyond fp16's range the fp16 dot overflows and the tf32 one does not
    big = u * 1e6
    assert not math.isfinite(O.dot(big, v, O.F16))
    assert O.dot(big, v, O.TF32) == O.dot(tf32_via_fp16(big), tf32_via_fp16(v), O.F32)


def test_action_encoding():
    assert O.action(O.TF32, O.F64, O.F64) == 128 + 25 * 4 + 5 * 3 + 3
    assert O.action(O.BF16, O.F32, O.F32) == 16 + 8 + 2       # no tf32: the 0..63 code
    for a in range(64):
        assert O.act_decode(a) == ((a >> 4) & 3, (a >> 2) & 3, a & 3)
    for a in range(64, 80):
        assert O.act_decode(a) == (O.Q52, (a >> 2) & 3, a & 3)
    digits = [O.F16, O.BF16, O.F32, O.F64, O.TF32]
    for ds in range(5):
        for dd in range(5):
            for da in range(5):
                f = (digits[ds], digits[dd], digits[da])
                a = O.action(*f)
                assert O.act_decode(a) == f
                assert (a >= 128) == (4 in (ds, dd, da))


def test_tf32_action_cost_in_the_reward():
    """C1: c(tf32) = 0.8 (section 5).  One fp64-CG iteration on a 2x2 system
    under action (tf32 SpMV, fp64 dot, fp64 update): the reward is
    -log10 rho_1 - 0.1 (0.8 + 2 + 2)."""
    A = W.CSR(2, np.array([0, 1, 2], np.int32), np.array([0, 1], np.int32), np.array([1.0, 2.0]))
    b = np.array([1.0, 1.0])
    a = O.action(O.TF32, O.F64, O.F64)
    pol = O.OraclePolicy(fixed_action=a, cost="C1")
    _, info = O.cg(A, b, tol=1e-300, maxit=1, policy=pol, replace_period=50, roll_cap=4)
    want = -math.log10(info["rho"][1]) - 0.1 * (0.8 + 2.0 + 2.0)
    assert abs(pol.reward(a, info["rho"][1], False) - want) <= 1e-12 * abs(want)
    assert abs(pol.reward(a, info["rho"][1], False) - pol.reward(63, info["rho"][1], False) - 0.1 * 1.2) < 1e-12


def test_five_format_tables_greedy_by_hand():
    """nfmt 5, per_op 2: Q_0 = (0, 0, 0, 0, 1) picks tf32 for the SpMV, Q_1 =
    (0, 0, 2, 0, 1) fp32 for the dot, the updates stay fp64: action
    128 + 25*4 + 5*2 + 3.  With per_op 1, Q_2 = (0, 3, 0, 0, 0) adds bf16
    updates."""
    A = W.laplacian_2d(6)
    b = W.rhs(A.n, 1)
    q = np.zeros((100, 64))
    q[0, 0:5], q[0, 5:10], q[0, 10:15] = (0, 0, 0, 0, 1), (0, 0, 2, 0, 1), (0, 3, 0, 0, 0)
    _, info = O.cg(A, b, tol=1e-8, maxit=1, policy=O.OraclePolicy(kind=O.POL_QTABLE, q=q, per_op=2, nfmt=5),
                   replace_period=50)
    assert info["actions"][0] == 128 + 100 + 10 + 3
    _, info = O.cg(A, b, tol=1e-8, maxit=1, policy=O.OraclePolicy(kind=O.POL_QTABLE, q=q, per_op=1, nfmt=5),
                   replace_period=50)
    assert info["actions"][0] == 128 + 100 + 10 + 1


def test_five_format_update_and_draws_by_hand():
    """Training with epsilon 0 on the 2x2 system: the chosen entries of Q_0 and
    Q_1 (columns 5 j + digit) move toward R + 0.9 max; epsilon 1: the digits
    are floor(5 u) from streams 3 and 5."""
    A = W.CSR(2, np.array([0, 1, 2], np.int32), np.array([0, 1], np.int32), np.array([1.0, 2.0]))
    b = np.array([1.0, 1.0])
    q0 = np.zeros((100, 64))
    q0[0, 4], q0[0, 7] = 1.0, 1.0              # Q_0: tf32, Q_1: fp32
    pol = O.OraclePolicy(kind=O.POL_QTRAIN, q=q0, epsilon=0.0, cost="C1", per_op=2, nfmt=5)
    _, info = O.cg(A, b, tol=1e-8, maxit=1, policy=pol, replace_period=50)
    a = 128 + 25 * 4 + 5 * 2 + 3
    assert info["actions"].tolist() == [a]
    R = -math.log10(info["rho"][1]) - 0.1 * (0.8 + 1.0 + 2.0)
    for c in (4, 7):
        assert abs(pol.q[0, c] - (1.0 + 0.1 * (R + 0.9 * 1.0 - 1.0))) < 1e-12
    assert np.count_nonzero(pol.q != q0) == 2

    L = W.laplacian_2d(16)
    bl = W.rhs(L.n, 2)
    pol = O.OraclePolicy(kind=O.POL_QTRAIN, epsilon=1.0, seed=11, episode=4, per_op=2, nfmt=5)
    _, info = O.cg(L, bl, tol=1e-8, maxit=30, policy=pol, replace_period=50, fallback=True)
    k = info["iters"] if info["fallback_at"] < 0 else info["fallback_at"]
    digits = [O.F16, O.BF16, O.F32, O.F64, O.TF32]
    want = [O.action(digits[int(O.uniform(11, 4, i, 3) * 5)], digits[int(O.uniform(11, 4, i, 5) * 5)], O.F64)
            for i in range(k)]
    assert info["actions"][:k].tolist() == want


def test_tf32_spmv_solve_equals_fp32_spmv_solve_on_an_integer_stencil():
    """The 3D Laplacian's entries are exact in tf32 and fp32, so the whole
    solve with a tf32 SpMV is the fp32-SpMV solve, bit for bit."""
    A = W.laplacian_3d(10)
    b = W.rhs(A.n, 5)
    x1, i1 = O.cg(A, b, tol=1e-10, maxit=500, policy=O.OraclePolicy(fixed_action=O.action(O.TF32, O.F64, O.F64)),
                  replace_period=50)
    x0, i0 = O.cg(A, b, tol=1e-10, maxit=500, policy=O.OraclePolicy(fixed_action=O.action(O.F32, O.F64, O.F64)),
                  replace_period=50)
    k = i0["iters"]
    assert i1["iters"] == k and np.array_equal(i1["rho"][:k + 1], i0["rho"][:k + 1]) and np.array_equal(x1, x0)
