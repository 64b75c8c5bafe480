"""Pins for the oracle's solver rules that the paper leaves to a reading:
the state's stagnation flag, the true-residual stagnation rule that triggers
the fp64 fallback, the tier switch (fold and re-round), the terminal reward of
a breakdown with its rollout row, and the bootstrapped update at truncation
(section 4.1's Q update; Algorithm 1).  Every expected value is worked by hand
from the definitions in the comments, or comes from an independent library
(numpy's float32 rounding), never from the oracle's own output.  CPU only."""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W


# ---------------------------------------------------------------- stag_k
def test_stag_flag_hand_history():
    # stag_k = [k >= W and rho_k >= rho_{k-W}]
    # W = 3 on rho = 1.0 .9 .8 .9 .9 .95 .5 .5:
    #   k < 3: 0;  k=3: .9 >= 1.0 no;  k=4: .9 >= .9 yes (equality counts);
    #   k=5: .95 >= .8 yes;  k=6: .5 >= .9 no;  k=7: .5 >= .9 no
    # (a window of W-1 flags k=3, a window of W+1 misses k=4, a strict
    #  comparison misses k=4, a reversed one flags k=3)
    h = [1.0, 0.9, 0.8, 0.9, 0.9, 0.95, 0.5, 0.5]
    assert [O.stag_flag(h, k, 3) for k in range(8)] == [0, 0, 0, 0, 1, 1, 0, 0]
    # W = 2 on rho = .5 .6 .7: k=1 has rho_1 >= rho_0 but k < W, so 0; k=2: .7 >= .5
    assert [O.stag_flag([0.5, 0.6, 0.7], k, 2) for k in range(3)] == [0, 0, 1]
    # W = 1 on a flat history: every k >= 1 is stagnant
    assert [O.stag_flag([0.3, 0.3, 0.3], k, 1) for k in range(3)] == [0, 1, 1]


# ---------------------------------------------------------------- m-2 stagnation rule
def first_firing(log):
    """First replacement m (1-based since the start) where the pinned rule fires."""
    for m in range(1, len(log) + 1):
        last3 = [log[m - 3] if m >= 3 else 0.0, log[m - 2] if m >= 2 else 0.0, log[m - 1]]
        if O.stagnated(m, last3):
            return m
    return None


def test_stagnation_rule_hand_logs():
    # fires at replacement m >= 3 when rho_true(m) >= rho_true(m-2)
    # log 1e-2 5e-3 6e-3 4e-3 7e-3: m=3: 6e-3 >= 1e-2 no; m=4: 4e-3 >= 5e-3 no;
    # m=5: 7e-3 >= 6e-3 yes  -> 5   (an m-1 rule would fire at m=3)
    assert first_firing([1e-2, 5e-3, 6e-3, 4e-3, 7e-3]) == 5
    # equality counts: 1e-2 5e-3 1e-2 -> m=3: 1e-2 >= 1e-2 yes
    assert first_firing([1e-2, 5e-3, 1e-2]) == 3
    # a steady decrease never fires
    assert first_firing([10.0 ** -j for j in range(1, 12)]) is None
    # m = 2 never fires, even when rho_true(2) exceeds rho_true(1)
    assert not O.stagnated(2, [0.0, 1e-3, 5e-3])
    assert not O.stagnated(1, [0.0, 0.0, 5e-3])


def test_stagnation_fallback_in_a_solve():
    """bf16 everywhere on a 32x32 Laplacian: the true residuals at the
    replacements (every 50 iterations) are about 7.54e-2, 4.11e-2, 3.76e-2,
    3.54e-2, 3.55e-2, 3.73e-2.  The rule first fires at m = 6 (3.73e-2 >= 3.54e-2),
    so the solve falls back at k = 300; an m-1 rule would fire at m = 5
    (3.55e-2 >= 3.54e-2), k = 250."""
    A = W.laplacian_2d(32)
    b = W.rhs(A.n, 2)
    pol = O.OraclePolicy(fixed_action=16 * 1 + 4 * 1 + 1)
    x, info = O.cg(A, b, tol=1e-8, maxit=3000, policy=pol, replace_period=50, fallback=True)
    rep = info["rep_rho"]
    assert info["rep_k"][:6].tolist() == [50, 100, 150, 200, 250, 300]
    assert first_firing(list(rep[:6])) == 6
    assert rep[4] >= rep[3]                      # the m-1 reading would have fired at m = 5
    assert info["fallback_at"] == 300 and info["status"] == 2
    assert info["flags"][299] & O.FL_FALLBACK
    assert not np.any(info["flags"][:299] & O.FL_FALLBACK)
    assert np.all(info["actions"][300:] == 63)   # fp64 CG after the restart
    assert info["relres_true"] <= 1e-8


# ---------------------------------------------------------------- tier switch
def switching_table(first, then):
    """Greedy table whose action is `first` in iteration bin 0 (k < 200) and
    `then` afterwards, whatever the residual bin and flag."""
    q = np.zeros((100, 64))
    for s in range(100):
        i = (s // 2) % 5
        q[s, first if i == 0 else then] = 1.0
    return q


def test_tier_switch_fp32_to_fp64():
    """The switch is decided after iteration 199, so iterations 0..199 are the
    fp32 solve's; widening r and p to fp64 changes no value."""
    A = W.laplacian_2d(64)
    b = W.rhs(A.n, 1)
    kw = dict(tol=1e-13, maxit=202, replace_period=0, dump=202)
    _, sw = O.cg(A, b, policy=O.OraclePolicy(kind=O.POL_QTABLE, q=switching_table(42, 63)), **kw)
    _, f32 = O.cg(A, b, policy=O.OraclePolicy(fixed_action=42), **kw)
    assert sw["actions"][:200].tolist() == [42] * 200 and sw["actions"][200:].tolist() == [63, 63]
    for key in ("r", "p"):
        assert np.array_equal(sw["dump"][key][:201], f32["dump"][key][:201])
    assert np.array_equal(sw["dump"]["r"][200], sw["dump"]["r"][200].astype(np.float32).astype(np.float64))
    assert [k for k in range(202) if sw["flags"][k] & O.FL_SWITCH] == [199]


def test_tier_switch_fp64_to_fp32_rerounds():
    """Going from fp64 to fp32 vectors, r and p are rounded to fp32 (round to
    nearest even, here numpy's float32 cast) right after the direction update
    of iteration 199: iteration 200 starts from the fp64 solve's r_200 and
    p_200 rounded."""
    A = W.laplacian_2d(64)
    b = W.rhs(A.n, 1)
    kw = dict(tol=1e-13, maxit=202, replace_period=0, dump=202)
    _, sw = O.cg(A, b, policy=O.OraclePolicy(kind=O.POL_QTABLE, q=switching_table(63, 42)), **kw)
    _, f64 = O.cg(A, b, policy=O.OraclePolicy(fixed_action=63), **kw)
    for key in ("r", "p"):
        assert np.array_equal(sw["dump"][key][:200], f64["dump"][key][:200])
        want = f64["dump"][key][200].astype(np.float32).astype(np.float64)
        assert np.array_equal(sw["dump"][key][200], want)
        assert not np.array_equal(want, f64["dump"][key][200])   # the rounding did something
    assert [k for k in range(202) if sw["flags"][k] & O.FL_SWITCH] == [199]


# ---------------------------------------------------------------- breakdown reward
def indefinite_2x2():
    # [[1, 2], [2, 1]]: eigenvalues 3 and -1, positive diagonal
    return W.CSR(2, np.array([0, 2, 4], np.int32), np.array([0, 1, 0, 1], np.int32),
                 np.array([1.0, 2.0, 2.0, 1.0]))


def test_breakdown_terminal_reward_and_rollout_row():
    """b = (1, -1): r_0 = p_0 = b, q = A p = (-1, 1), nu = p.q = -2 < 0, so
    iteration 0 breaks down.  An all-zero table picks action 0 (fp16 x3, cost
    3 * 0.8 = 2.4 under C1); the breakdown is terminal with reward
    -0.1 * 2.4 - 10 = -10.24, and Q[s_0, 0] = 0 + 0.1 * (-10.24 - 0) = -1.024.
    s_0: k = 0, rho_0 = 1 (bin 0), no stagnation -> state 0.  Its features: the
    eight log10 rho lags of rho_0 = 1 are 0, the difference 0, k / 1000 = 0,
    stag 0, log10 of the last true rho = 0, (k mod R) / R = 0, and the previous
    action (fp64 x3 at the start) gives 3/3 three times."""
    A = indefinite_2x2()
    b = np.array([1.0, -1.0])
    pol = O.OraclePolicy(kind=O.POL_QTRAIN, epsilon=0.0, cost="C1")
    _, info = O.cg(A, b, tol=1e-8, maxit=10, policy=pol, replace_period=50, roll_cap=8)
    assert info["status"] == 3 and info["iters"] == 0
    assert abs(pol.q[0, 0] - (-1.024)) < 1e-12
    assert np.count_nonzero(pol.q) == 1
    ro = info["rollouts"]
    assert len(ro["act"]) == 1 and ro["act"][0] == 0 and ro["done"][0] == 1
    assert ro["rew"][0] == np.float32(-10.24)
    want_f = np.array([0.0] * 13 + [1.0, 1.0, 1.0], np.float32)
    assert np.array_equal(ro["feat"][0], want_f) and np.array_equal(ro["next"][0], want_f)
    # with the fallback: the fp64 restart breaks down the same way; the policy
    # no longer acts, so nothing more is logged or learned
    pol2 = O.OraclePolicy(kind=O.POL_QTRAIN, epsilon=0.0, cost="C1")
    _, info2 = O.cg(A, b, tol=1e-8, maxit=10, policy=pol2, replace_period=50, fallback=True, roll_cap=8)
    assert info2["status"] == 3 and info2["fallback_at"] == 0
    assert len(info2["rollouts"]["act"]) == 1 and abs(pol2.q[0, 0] - (-1.024)) < 1e-12


# ---------------------------------------------------------------- truncation bootstrap
def test_truncation_at_maxit_bootstraps():
    """A = diag(1, 2), b = (1, 1), maxit = 1, a table with Q[0, 42] = 1 (so the
    greedy action is fp32 x3, cost 3.0 under C1).  One fp32 iteration:
    q = (1, 2), nu = 3, sigma = 2, alpha = 2/3; with a = fl32(2/3),
    r_1 = (fl32(1 - a), fl32(1 - 2a)) = (1 - a, 1 - 2a) exactly; sigma' = the
    fp32 sum of the fp32 squares; rho_1 = sqrt(sigma') / sqrt(2), about 1/3,
    bin 0, k = 1 < W: state 0 again.  The episode is cut at maxit, which is not
    terminal (section 4.1's update with the bootstrap term):
    Q[0, 42] = 1 + 0.1 * (R + 0.9 * max_a Q[0, a] - 1), max = 1 (read before
    the update), R = -log10 rho_1 - 0.1 * 3.0."""
    A = W.CSR(2, np.array([0, 1, 2], np.int32), np.array([0, 1], np.int32), np.array([1.0, 2.0]))
    b = np.array([1.0, 1.0])
    q0 = np.zeros((100, 64))
    q0[0, 42] = 1.0
    pol = O.OraclePolicy(kind=O.POL_QTRAIN, q=q0, epsilon=0.0, cost="C1")
    _, info = O.cg(A, b, tol=1e-8, maxit=1, policy=pol, replace_period=50)
    assert info["status"] == 1 and info["iters"] == 1 and info["actions"].tolist() == [42]
    a = np.float32(2.0 / 3.0)
    r1 = np.array([np.float32(1.0) - a, np.float32(1.0) - np.float32(2.0) * a], np.float32)
    assert r1[0] == np.float32(5592405 / 2 ** 24) and r1[1] == np.float32(-5592406 / 2 ** 24)
    sig = np.float32(r1[0] * r1[0]) + np.float32(r1[1] * r1[1])
    rho1 = math.sqrt(float(sig)) / math.sqrt(2.0)
    assert info["rho"][1] == rho1
    R = -math.log10(rho1) - 0.1 * 3.0
    boot = 1.0 + 0.1 * (R + 0.9 * 1.0 - 1.0)
    assert abs(pol.q[0, 42] - boot) < 1e-12
    assert abs(pol.q[0, 42] - (1.0 + 0.1 * (R - 1.0))) > 1e-3   # the terminal form differs


# ---------------------------------------------------------------- decision period
def test_decision_period_one_update_per_decision():
    """Two eigencomponents: fp64 CG converges in two iterations.  With D = 1 the
    two transitions update Q[s0, 63] and Q[s1, 63] (section 4.1).  With D = 8
    the decision taken at k = 0 holds through both iterations and ends at
    convergence: one terminal update of Q[s0, 63] toward
    R = -log10 rho_2 - 0.1 * (6.0 * 2) + 10, the cost of both iterations."""
    A = W.laplacian_2d(8)
    ev, V = np.linalg.eigh(A.to_dense())
    b = V[:, 2] + 0.5 * V[:, 40]
    q0 = np.zeros((100, 64))
    q0[:, 63] = 0.25
    pol = O.OraclePolicy(kind=O.POL_QTRAIN, q=q0, epsilon=0.0, cost="C1", decision_period=8)
    x, info = O.cg(A, b, tol=1e-10, maxit=5, policy=pol, replace_period=50)
    assert info["status"] == 0 and info["iters"] == 2
    rho2 = info["rho"][2]
    s0 = pol.state(0, 1.0, 0)
    R = (16.0 if rho2 <= 1e-16 else -math.log10(rho2)) - 0.1 * (6.0 * 2) + 10.0
    assert abs(pol.q[s0, 63] - (0.25 + 0.1 * (R - 0.25))) < 1e-12
    assert np.count_nonzero(pol.q != q0) == 1


def test_decision_period_holds_the_action_and_logs_one_row_per_decision():
    """A greedy table whose best action differs in every state: with D = 5 the
    action changes only at k = 0, 5, 10, ...; with rollout logging each
    decision leaves one row, whose reward charges its 5 iterations."""
    A = W.laplacian_2d(20)
    b = W.rhs(A.n, 7)
    rng = np.random.default_rng(3)
    q = rng.standard_normal((100, 64))
    q[:, 42] += 5.0                      # fp32 actions mostly, so the solve runs long
    q[::3, 26] += 7.0
    pol = O.OraclePolicy(kind=O.POL_QTABLE, q=q, decision_period=5)
    x, info = O.cg(A, b, tol=1e-8, maxit=60, policy=pol, replace_period=50, roll_cap=100)
    acts = info["actions"]
    k = info["iters"]
    for i in range(1, k):
        if i % 5:
            assert acts[i] == acts[i - 1]
    ro = info["rollouts"]
    assert len(ro["act"]) == (k + 4) // 5
    # the first decision's reward: accuracy at rho_5 minus 5 iterations of its cost
    c = {0: 0.8, 1: 0.6, 2: 1.0, 3: 2.0}
    a0 = int(acts[0])
    cost = c[(a0 >> 4) & 3] + c[(a0 >> 2) & 3] + c[a0 & 3]
    want = -math.log10(info["rho"][5]) - 0.1 * cost * 5
    assert abs(float(ro["rew"][0]) - want) <= 1e-5 * max(1.0, abs(want))


# ---------------------------------------------------------------- one Q-table per operation
def test_per_op_greedy_action():
    """Q_0 = (0, 3, 1, 2), Q_1 = (5, 5, 0, 0) (a tie: the lower format),
    Q_2 = (0, 0, 0, 1): the action is 16*1 + 4*0 + 3 = 19 (bf16 SpMV, fp16 dot,
    fp64 update)."""
    A = W.laplacian_2d(6)
    b = W.rhs(A.n, 1)
    q = np.zeros((100, 64))
    q[0, 0:4], q[0, 4:8], q[0, 8:12] = (0, 3, 1, 2), (5, 5, 0, 0), (0, 0, 0, 1)
    q[0, 19 + 20] = 100.0                  # the joint reading of the row would pick 39
    pol = O.OraclePolicy(kind=O.POL_QTABLE, q=q, per_op=1)
    _, info = O.cg(A, b, tol=1e-8, maxit=1, policy=pol, replace_period=50)
    assert info["actions"][0] == 19
    _, info = O.cg(A, b, tol=1e-8, maxit=1, policy=O.OraclePolicy(kind=O.POL_QTABLE, q=q), replace_period=50)
    assert info["actions"][0] == 39


def test_per_op_truncation_update_by_hand():
    """The 2x2 system of test_truncation_at_maxit_bootstraps with one table per
    operation, each preferring fp32 (Q_j(0, fp32) = 1): one fp32 iteration, then
    the cut at maxit updates every table's fp32 entry toward R + 0.9 * 1 (the
    bootstrap from state 0 again): Q_j(0, fp32) = 1 + 0.1 (R + 0.9 - 1)."""
    A = W.CSR(2, np.array([0, 1, 2], np.int32), np.array([0, 1], np.int32), np.array([1.0, 2.0]))
    b = np.array([1.0, 1.0])
    q0 = np.zeros((100, 64))
    q0[0, [2, 6, 10]] = 1.0
    pol = O.OraclePolicy(kind=O.POL_QTRAIN, q=q0, epsilon=0.0, cost="C1", per_op=1)
    _, info = O.cg(A, b, tol=1e-8, maxit=1, policy=pol, replace_period=50)
    assert info["actions"].tolist() == [42]
    R = -math.log10(info["rho"][1]) - 0.1 * 3.0
    want = 1.0 + 0.1 * (R + 0.9 * 1.0 - 1.0)
    for c in (2, 6, 10):
        assert abs(pol.q[0, c] - want) < 1e-12
    assert np.count_nonzero(pol.q != q0) == 3


def test_per_op_exploration_draws():
    """epsilon = 1: every operation draws its format from its own stream,
    floor(4 u) with u = uniform(seed, episode, k, 3 + 2 j)."""
    A = W.laplacian_2d(16)
    b = W.rhs(A.n, 2)
    pol = O.OraclePolicy(kind=O.POL_QTRAIN, epsilon=1.0, seed=11, episode=4, per_op=1)
    x, info = O.cg(A, b, tol=1e-8, maxit=30, policy=pol, replace_period=50, fallback=True)
    k = info["iters"] if info["fallback_at"] < 0 else info["fallback_at"]
    want = [16 * int(O.uniform(11, 4, i, 3) * 4) + 4 * int(O.uniform(11, 4, i, 5) * 4) + int(O.uniform(11, 4, i, 7) * 4)
            for i in range(k)]
    assert info["actions"][:k].tolist() == want


def test_per_op_fp64_updates_greedy_and_update_by_hand():
    """per_op = 2: tables for the SpMV and the dot only, the updates in fp64
    whatever Q_2 holds.  Q_0 prefers bf16, Q_1 fp32, Q_2 fp16: the action is
    16*1 + 4*2 + 3 = 27.  In training with epsilon 0 the cut at maxit = 1
    moves the two tables' chosen entries toward R + 0.9 max Q_j(0, .), and
    Q_2 is left as it was."""
    A = W.CSR(2, np.array([0, 1, 2], np.int32), np.array([0, 1], np.int32), np.array([1.0, 2.0]))
    b = np.array([1.0, 1.0])
    q0 = np.zeros((100, 64))
    q0[0, 1], q0[0, 6], q0[0, 8] = 1.0, 1.0, 5.0
    _, info = O.cg(A, b, tol=1e-8, maxit=1, policy=O.OraclePolicy(kind=O.POL_QTABLE, q=q0, per_op=2),
                   replace_period=50)
    assert info["actions"].tolist() == [27]
    pol = O.OraclePolicy(kind=O.POL_QTRAIN, q=q0, epsilon=0.0, cost="C1", per_op=2)
    _, info = O.cg(A, b, tol=1e-8, maxit=1, policy=pol, replace_period=50)
    assert info["actions"].tolist() == [27]
    R = -math.log10(info["rho"][1]) - 0.1 * (0.6 + 1.0 + 2.0)
    for c in (1, 6):
        assert abs(pol.q[0, c] - (1.0 + 0.1 * (R + 0.9 * 1.0 - 1.0))) < 1e-12
    assert np.count_nonzero(pol.q != q0) == 2 and pol.q[0, 8] == 5.0


def test_per_op_fp64_updates_exploration_draws():
    """per_op = 2 with epsilon = 1: the SpMV and the dot draw from streams 3
    and 5, the update stays fp64 and stream 7 is never read."""
    A = W.laplacian_2d(16)
    b = W.rhs(A.n, 2)
    pol = O.OraclePolicy(kind=O.POL_QTRAIN, epsilon=1.0, seed=11, episode=4, per_op=2)
    x, info = O.cg(A, b, tol=1e-8, maxit=30, policy=pol, replace_period=50, fallback=True)
    k = info["iters"] if info["fallback_at"] < 0 else info["fallback_at"]
    want = [16 * int(O.uniform(11, 4, i, 3) * 4) + 4 * int(O.uniform(11, 4, i, 5) * 4) + 3 for i in range(k)]
    assert info["actions"][:k].tolist() == want


# ---------------------------------------------------------------- rho in fp64
def test_rho_fp64_by_hand():
    """A = diag(1, 4), b = 2^-14 (1, 1), action 51 (fp64 SpMV and updates, fp16
    dots).  By hand: nu = 5 s^2 (exact in every format), alpha = rd(2/5),
    r_1 = s (rd(1 - alpha), rd(1 - 4 alpha)).  With rho_fp64, rho_1 is the fp64
    norm of r_1 over ||b|| = s sqrt(2); without it, rho_1 comes from the fp16
    dot, whose operands 0.6 s fall in fp16's subnormal range (steps of 2^-24).
    sigma' is dot_fp16(r, r) either way, so the iterates agree bit for bit."""
    s = 2.0 ** -14
    A = W.CSR(2, np.array([0, 1, 2], np.int32), np.array([0, 1], np.int32), np.array([1.0, 4.0]))
    b = np.array([s, s])
    pol = O.OraclePolicy(fixed_action=51)
    alpha = 2.0 / 5.0
    a, c = 1.0 - alpha, 1.0 - 4.0 * alpha
    want64 = np.sqrt(a * a + c * c) / np.sqrt(2.0)
    h = [abs(float(np.float16(v * s))) * 2.0 ** 24 for v in (a, c)]   # integers: fp16 subnormal units
    assert all(v == int(v) for v in h)
    want16 = np.sqrt(h[0] ** 2 + h[1] ** 2) / np.sqrt(2.0) / 1024.0
    x1, i1 = O.cg(A, b, tol=1e-300, maxit=2, policy=pol, replace_period=50, rho_fp64=1)
    x0, i0 = O.cg(A, b, tol=1e-300, maxit=2, policy=pol, replace_period=50, rho_fp64=0)
    assert i1["rho"][1] == want64 and i0["rho"][1] == want16 and want16 != want64
    assert np.array_equal(x1, x0) and i1["iters"] == i0["iters"] == 2


@pytest.mark.parametrize("act", [63, 16 * 1 + 4 * 3 + 2])
def test_rho_fp64_changes_nothing_with_fp64_dots(act):
    """With the dot already in fp64 the two readings of rho coincide."""
    A = W.laplacian_2d(12)
    b = W.rhs(A.n, 3)
    pol = O.OraclePolicy(fixed_action=act)
    x1, i1 = O.cg(A, b, tol=1e-9, maxit=300, policy=pol, replace_period=50, rho_fp64=1)
    x0, i0 = O.cg(A, b, tol=1e-9, maxit=300, policy=pol, replace_period=50)
    k = i0["iters"]
    assert i1["iters"] == k and np.array_equal(i1["rho"][:k + 1], i0["rho"][:k + 1]) and np.array_equal(x1, x0)


# ---------------------------------------------------------------- the paper's termination
def test_paper_termination_needs_ten_iterations():
    """An eigenvector right-hand side: fp64 CG's recursive residual falls below
    1e-6 after one iteration.  Section 5's rule (rho < tol with k >= 10) runs
    to exactly k = 10; the default rule stops at the first replacement (k = 1).
    Either way the reported relres is the final x's true residual."""
    A = W.laplacian_2d(8)
    ev, V = np.linalg.eigh(A.to_dense())
    b = V[:, 5].copy()
    x1, i1 = O.cg(A, b, tol=1e-6, maxit=100, stop_rule=1)
    x0, i0 = O.cg(A, b, tol=1e-6, maxit=100)
    assert i0["iters"] == 1 and i1["iters"] == 10 and i1["status"] == 0
    assert i1["rho"][1] < 1e-6 and np.all(i1["rho"][1:11] < 1e-6)
    r = O.residual(A, b, x1)
    assert i1["relres_true"] == np.sqrt(O.dot(r, r, O.F64)) / np.sqrt(O.dot(b, b, O.F64))
    assert abs(i1["relres_true"] - np.linalg.norm(b - A.to_dense() @ x1) / np.linalg.norm(b)) <= 1e-15
    assert i1["n_replace"] == 0


def test_paper_termination_on_the_recursive_residual():
    """bf16 updates: the recursive residual leaves the true one; the paper's
    rule stops at the first k >= 10 with rho_k < tol on the recursion, whatever
    the true residual (which the result still reports)."""
    A = W.laplacian_2d(30)
    b = W.rhs(A.n, 5)
    x, info = O.cg(A, b, tol=1e-6, maxit=3000, policy=O.OraclePolicy(fixed_action=16 * 1 + 4 * 1 + 1),
                   replace_period=0, stop_rule=1)
    rho = info["rho"]
    k = info["iters"]
    assert info["status"] == 0 and k >= 10 and rho[k] < 1e-6
    assert not any(rho[j] < 1e-6 for j in range(10, k))
    r = O.residual(A, b, x)
    assert info["relres_true"] == np.sqrt(O.dot(r, r, O.F64)) / np.sqrt(O.dot(b, b, O.F64))
