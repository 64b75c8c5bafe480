"""The library derives the residual-bin thresholds of section 4.1 itself
(mpcg_residual_thresholds, pure host code): T_j is the double nearest to
10^(-E j / b_res) for eps_min = 10^-E.  Checked against the oracle's
independent decimal computation over a grid of (E, b_res), against the log
formula for the bin index, and for its argument checks.  Runs without a GPU."""
import math
import os

import numpy as np
import pytest

import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2504_14268_amd", "libmpcg.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libmpcg.so not built")


@pytest.mark.parametrize("E", [1, 2, 3, 5, 7, 8, 12, 16, 17, 23, 30, 64, 150, 300])
def test_thresholds_equal_decimal_nearest(E):
    import paper_2504_14268_amd as M

    for b_res in range(1, 18):
        got = list(M.residual_thresholds(b_res, float(f"1e-{E}")))
        assert got == O.residual_edges(b_res, E), (E, b_res)


def test_paper_default_thresholds():
    import paper_2504_14268_amd as M

    t = M.residual_thresholds(10, 1e-16)
    assert len(t) == 9 and t[4] == 1e-8          # 10^(-1.6*5) = 1e-8 exactly representable target
    assert all(a > b for a, b in zip(t, t[1:]))
    for j, v in enumerate(t, 1):
        # the real boundary 10^(-1.6 j) lies within half an ulp of T_j
        assert abs(math.log10(v) + 1.6 * j) < 1e-15 * 4


def test_bins_match_the_floor_formula_off_the_boundaries():
    import paper_2504_14268_amd as M

    t = M.residual_thresholds(10, 1e-16)
    rng = np.random.default_rng(4)
    for rho in 10.0 ** rng.uniform(-17, 1, 3000):
        if min(abs(math.log10(rho) + 1.6 * j) for j in range(1, 10)) < 1e-9:
            continue
        j_formula = min(max(math.floor(-math.log10(max(rho, 1e-16)) / 1.6), 0), 9)
        assert int(np.sum(rho <= t)) == j_formula


@pytest.mark.parametrize("b_res,eps", [(10, 2e-16), (10, 1e-16 * (1 + 2 ** -52)), (10, 0.0), (10, 1.0),
                                        (10, float("nan")), (10, -1e-16), (0, 1e-16), (18, 1e-16),
                                        (10, 1e-301)])
def test_thresholds_reject_bad_arguments(b_res, eps):
    import paper_2504_14268_amd as M

    with pytest.raises(M.MPCGError):
        M.residual_thresholds(b_res, eps)
