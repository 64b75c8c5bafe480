"""Pins for the oracle's q52 (Table 1's quarter precision; 5 exponent bits,
t = 3) matrix storage: Table 1's row, every bit pattern as a fixed point,
rounding against brute force over the finite set and against torch's
float8_e5m2 (an independent implementation), the per-row scale, and the SpMV
on integer stencils (exact) and random matrices (within its error bound).
CPU only."""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
import workloads as W


def q52_values():
    """All 256 bit patterns decoded from the format's definition: sign, 5-bit
    biased exponent (bias 15), 2 fraction bits; exponent 0 is subnormal
    (2^-14 * f/4), exponent 31 is inf/NaN."""
    out = []
    for b in range(256):
        s = -1.0 if b & 0x80 else 1.0
        e = (b >> 2) & 0x1F
        f = b & 3
        if e == 31:
            out.append(s * math.inf if f == 0 else math.nan)
        elif e == 0:
            out.append(s * 2.0 ** -14 * f / 4)
        else:
            out.append(s * 2.0 ** (e - 15) * (1 + f / 4))
    return out


def test_table1_q52_row():
    # u = 1.25e-1, x_min = 6.10e-5, x_max = 5.73e4, e_min = -14, e_max = 15, t read as 3
    t, emin, emax = 3, -14, 15
    assert 2.0 ** -t == 0.125
    assert float(f"{2.0 ** emin:.2e}") == 6.10e-5
    big = (2.0 - 2.0 ** (1 - t)) * 2.0 ** emax
    assert big == 57344.0 and float(f"{big:.2e}") == 5.73e4
    assert O.rd(big, O.Q52)[0] == big
    assert O.rd(2.0 ** emin, O.Q52)[0] == 2.0 ** emin
    assert O.rd(1.0 + 0.125, O.Q52)[0] == 1.0                 # u: the tie above 1 rounds to even
    assert O.rd(1.0 + 0.125 * 1.001, O.Q52)[0] == 1.25
    assert O.rd(big + 4096.0, O.Q52)[0] == math.inf           # tie above x_max overflows
    assert O.rd(big + 4095.0, O.Q52)[0] == big
    assert O.rd(2.0 ** -17, O.Q52)[0] == 0.0                  # half the smallest subnormal: to even (0)
    assert O.rd(3 * 2.0 ** -18, O.Q52)[0] == 2.0 ** -16


def test_every_pattern_is_a_fixed_point():
    vals = np.array([v for v in q52_values() if math.isfinite(v)])
    assert len(set(vals.tolist())) == 247               # 248 finite patterns, +0 and -0 compare equal
    assert np.array_equal(O.rd(vals, O.Q52), vals)


def brute_nearest_even(x, finite):
    """Nearest finite q52 value, ties to the one with an even last fraction bit;
    beyond x_max + half an ulp: infinity."""
    if abs(x) >= 57344.0 + 4096.0:
        return math.copysign(math.inf, x)
    best = None
    for b, v in finite:
        d = abs(Fraction(x) - Fraction(v))
        if best is None or d < best[0] or (d == best[0] and (b & 1) == 0 and (best[1] & 1) == 1):
            best = (d, b, v)
    return best[2] if best[2] != 0.0 else math.copysign(0.0, x)


def test_rounding_against_brute_force():
    finite = [(b, v) for b, v in enumerate(q52_values()) if math.isfinite(v) and not (b & 0x80)]
    rng = np.random.default_rng(52)
    xs = list(10.0 ** rng.uniform(-6, 5, 400)) + [0.0625 * 1.125, 1.375, 2.0 ** -16 * 1.5, 2.0 ** -16 * 0.5,
                                                  61439.9, 61440.0, 5e-6]
    mids = [(a + b) / 2 for (_, a), (_, b) in zip(finite, finite[1:])]
    xs += mids
    for x in xs:
        for sx in (x, -x):
            want = brute_nearest_even(abs(sx), finite)
            want = math.copysign(want, sx) if want == want else want
            assert O.rd(sx, O.Q52)[0] == want, sx


def test_rounding_against_torch_float8_e5m2():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(3)
    x = np.concatenate([(rng.standard_normal(20000) * 10.0 ** rng.uniform(-7, 5, 20000)),
                        rng.uniform(-70000, 70000, 2000)]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.float8_e5m2).to(torch.float32).numpy().astype(np.float64)
    got = O.rd(x.astype(np.float64), O.Q52)
    assert np.array_equal(got, ref)


def test_q52_row_scale_and_shadow():
    A = W.random_spd(400, 11, spread=2.0)
    v, e = O.shadow_q52(A)
    s32, sb, sh, e16 = O.shadows(A)
    assert np.array_equal(e, e16)                        # the fp16 row exponents
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    scaled = A.val * 2.0 ** -e[rows].astype(np.float64)
    assert np.all(np.abs(scaled) <= 2.0 ** 15)
    assert np.array_equal(v, O.rd(scaled, O.Q52))


@pytest.mark.parametrize("tier", [0, 1])
def test_spmv_q52_laplacian_integer_exact(tier):
    """Stencil values 4, 6 and -1 are exact in q52 after the row scale, so with
    small integer p the q52 SpMV is the dense product exactly."""
    rng = np.random.default_rng(7)
    for A in (W.laplacian_2d(13), W.laplacian_3d(7)):
        p = rng.integers(-300, 300, A.n).astype(np.float64)
        assert np.array_equal(O.spmv(A, p, O.Q52, tier), A.to_dense() @ p)


def test_spmv_q52_error_bound_random():
    """|q_i - exact_i| <= u_q52 * sum |a p| (value rounding) + gamma_{m+1}(fp32) * sum |a p|
    (products, fma chain, output) + the subnormal quantum 2^-17 * 2^e_i per entry."""
    A = W.random_spd(300, 5, spread=1.0)
    rng = np.random.default_rng(8)
    p = rng.standard_normal(A.n).astype(np.float32).astype(np.float64)
    q = O.spmv(A, p, O.Q52, 1)
    _, e = O.shadow_q52(A)
    u32 = 2.0 ** -24
    for i in range(A.n):
        s, t = A.row_ptr[i], A.row_ptr[i + 1]
        m = t - s
        exact = float(sum(Fraction(float(a)) * Fraction(float(x)) for a, x in zip(A.val[s:t], p[A.col[s:t]])))
        absum = float(np.sum(np.abs(A.val[s:t] * p[A.col[s:t]])))
        g = (m + 1) * u32 / (1 - (m + 1) * u32)
        bound = (0.125 + g) * absum * 1.01 + 2.0 ** (-17 + int(e[i])) * float(np.sum(np.abs(p[A.col[s:t]])))
        assert abs(q[i] - exact) <= bound
