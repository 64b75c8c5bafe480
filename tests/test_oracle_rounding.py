"""Pins for the oracle's round-to-format (Table 1 formats) against Table 1,
exact rational arithmetic and two independent libraries (numpy float16, torch
bfloat16).  CPU only."""
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")
FMT = {"fp16": O.F16, "bf16": O.BF16, "fp32": O.F32, "fp64": O.F64}


def table1():
    rows = {}
    for line in open(os.path.join(GOLD, "table1_formats.txt")):
        if line.startswith("#") or not line.strip():
            continue
        name, u, xmin, xmax, t, emin, emax = line.split()
        rows[name] = (float(u), float(xmin), float(xmax), int(t), int(emin), int(emax))
    return rows


def sig3(x):
    return float(f"{x:.2e}")


@pytest.mark.parametrize("name", ["fp16", "bf16", "fp32", "fp64"])
def test_table1_constants(name):
    """Unit roundoff, smallest normal and largest finite value of each format, as
    the oracle realises them, print as Table 1 does."""
    u, xmin, xmax, t, emin, emax = table1()[name]
    f = FMT[name]
    one = 1.0
    # u = 2^-t: 1 + u is the tie between 1 and 1 + 2u and rounds to even (1).
    uu = 2.0 ** -t
    assert O.rd(one + uu, f)[0] == 1.0 or f == O.F64
    if f != O.F64:
        assert O.rd(one + uu * (1 + 2.0 ** -20), f)[0] == one + 2 * uu
        assert O.rd(one + uu * (1 - 2.0 ** -20), f)[0] == one
    assert sig3(uu) == u
    # smallest normal 2^emin is representable, and so is the largest finite value
    assert O.rd(2.0 ** emin, f)[0] == 2.0 ** emin
    assert sig3(2.0 ** emin) == xmin
    big = (2.0 - 2.0 ** (1 - t)) * 2.0 ** emax
    assert O.rd(big, f)[0] == big
    assert sig3(big) == xmax
    if f != O.F64:
        half_ulp = 2.0 ** (emax - t)
        assert O.rd(big + half_ulp, f)[0] == np.inf          # tie above x_max: overflow
        assert O.rd(big + half_ulp * 0.999, f)[0] == big
        assert O.rd(-(big + half_ulp), f)[0] == -np.inf


def test_fp16_all_patterns_roundtrip_and_numpy():
    """Every finite fp16 value is a fixed point; numpy's float64->float16
    conversion (an independent implementation) agrees on random doubles."""
    bits = np.arange(65536, dtype=np.uint16)
    h = bits.view(np.float16)
    fin = np.isfinite(h)
    x = h[fin].astype(np.float64)
    assert np.array_equal(O.rd(x, O.F16), x)
    rng = np.random.default_rng(0)
    for scale in (1e-9, 1e-6, 1e-3, 1.0, 1e3, 6e4, 7e4):
        y = rng.standard_normal(20000) * scale
        assert np.array_equal(O.rd(y, O.F16), y.astype(np.float16).astype(np.float64))


def test_bf16_all_patterns_roundtrip_and_torch():
    torch = pytest.importorskip("torch")
    bits = np.arange(65536, dtype=np.uint32) << 16
    x = bits.view(np.float32).astype(np.float64)
    x = x[np.isfinite(x)]
    assert np.array_equal(O.rd(x, O.BF16), x)
    rng = np.random.default_rng(1)
    for scale in (1e-40, 1e-30, 1.0, 1e30, 3e38):
        y32 = (rng.standard_normal(20000) * scale).astype(np.float32)
        ref = torch.from_numpy(y32).to(torch.bfloat16).to(torch.float64).numpy()
        assert np.array_equal(O.rd(y32.astype(np.float64), O.BF16), ref)


def test_fp32_matches_native_cast():
    rng = np.random.default_rng(2)
    for scale in (1e-44, 1e-40, 1e-10, 1.0, 1e30, 3.4e38):
        y = rng.standard_normal(20000) * scale
        assert np.array_equal(O.rd(y, O.F32), y.astype(np.float32).astype(np.float64))


def test_direct_rounding_from_fp64_not_via_fp32():
    """x just above the bf16 midpoint 1 + 2^-8: fp64 -> fp32 lands exactly on the
    midpoint (ties to 1.0), but direct rounding must go up to 1 + 2^-7."""
    x = 1.0 + 2.0 ** -8 + 2.0 ** -30
    assert O.rd(x, O.BF16)[0] == 1.0 + 2.0 ** -7
    assert O.rd(O.rd(x, O.F32)[0], O.BF16)[0] == 1.0
    y = 1.0 + 2.0 ** -11 + 2.0 ** -40
    assert O.rd(y, O.F16)[0] == 1.0 + 2.0 ** -10


def test_subnormals_ties_to_even():
    s = 2.0 ** -24                         # smallest fp16 subnormal
    assert O.rd(s / 2, O.F16)[0] == 0.0    # tie between 0 and s: even is 0
    assert O.rd(s / 2 * (1 + 2.0 ** -20), O.F16)[0] == s
    assert O.rd(1.5 * s, O.F16)[0] == 2 * s  # tie between s and 2s: even is 2s
    assert O.rd(2.5 * s, O.F16)[0] == 2 * s
    sb = 2.0 ** -133                       # smallest bf16 subnormal
    assert O.rd(1.5 * sb, O.BF16)[0] == 2 * sb
    assert O.rd(sb * 0.5, O.BF16)[0] == 0.0
    assert O.rd(-1.5 * s, O.F16)[0] == -2 * s
    assert np.isnan(O.rd(np.nan, O.F16)[0])
    assert O.rd(-np.inf, O.BF16)[0] == -np.inf


def round_fraction(fr: Fraction, t: int, emin: int, emax: int) -> float:
    """Exact rational round-to-nearest-even to a binary format (independent of the oracle)."""
    if fr == 0:
        return 0.0
    sign = -1 if fr < 0 else 1
    a = abs(fr)
    E = a.numerator.bit_length() - a.denominator.bit_length()
    if Fraction(2) ** E > a:
        E -= 1
    E = max(E, emin)
    q = Fraction(2) ** (E - t + 1)
    m = a / q
    fl = m.numerator // m.denominator
    rem = m - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        fl += 1
    y = fl * q
    if y > (2 - Fraction(2) ** (1 - t)) * Fraction(2) ** emax:
        return sign * float("inf")
    return sign * float(y)


def test_rounding_against_exact_rationals():
    rng = np.random.default_rng(3)
    fmts = [(O.F16, 11, -14, 15), (O.BF16, 8, -126, 127), (O.F32, 24, -126, 127)]
    xs = np.concatenate([rng.standard_normal(400) * 10.0 ** rng.integers(-8, 6, 400),
                         rng.standard_normal(100) * 1e-6])
    for f, t, emin, emax in fmts:
        got = O.rd(xs, f)
        ref = np.array([round_fraction(Fraction(float(v)), t, emin, emax) for v in xs])
        assert np.array_equal(got, ref)
