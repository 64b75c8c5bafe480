"""Pins for the oracle's policy machinery (section 4.1; Algorithms 1 and 2):
state discretisation at its boundaries and against the log formula, the reward
on hand-worked examples, tabular Q-learning updates worked by hand, the
published SplitMix64 vector behind the exploration draws, the decimal log and
GELU against the standard library, and the MLP forward against an independent
float64 evaluation.  CPU only."""
import math
import os

import numpy as np
import pytest

import oracle as O
import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_residual_edges_are_nearest_doubles():
    e = O.residual_edges()
    assert len(e) == 9 and e[4] == 1e-8
    for j, t in enumerate(e, 1):
        assert abs(math.log10(t) + 1.6 * j) < 1e-14
        assert all(a > b for a, b in zip(e, e[1:]))


def log_formula_bin(rho, k, stag, b_it=5, t_bin=1000, b_res=10, eps_min=1e-16):
    i = min(k // math.ceil(t_bin / b_it), b_it - 1)
    delta = -math.log10(eps_min) / b_res
    j = min(math.floor(-math.log10(max(rho, eps_min)) / delta), b_res - 1)
    j = max(j, 0)
    return (j * b_it + i) * 2 + int(stag)


def test_state_bins_boundaries():
    pol = O.OraclePolicy()
    e = O.residual_edges()
    for j, t in enumerate(e, 1):
        assert pol.state(0, t, 0) == 2 * 5 * j                      # at the edge: the lower bin
        assert pol.state(0, np.nextafter(t, 1.0), 0) == 2 * 5 * (j - 1)
        assert pol.state(0, np.nextafter(t, 0.0), 0) == 2 * 5 * j
    assert pol.state(0, 5.0, 0) == 0                                # rho > 1 clamps to bin 0
    assert pol.state(0, 1e-300, 0) == 2 * 5 * 9
    assert pol.state(0, 0.0, 1) == 2 * 5 * 9 + 1
    for k, ib in ((0, 0), (199, 0), (200, 1), (799, 3), (800, 4), (999, 4), (5000, 4)):
        assert pol.state(k, 0.5, 0) == 2 * ib
    rng = np.random.default_rng(0)
    for _ in range(2000):
        rho = 10.0 ** rng.uniform(-17, 1)
        k = int(rng.integers(0, 3000))
        stag = int(rng.integers(0, 2))
        if min(abs(math.log10(rho) + 1.6 * j) for j in range(1, 10)) < 1e-9:
            continue
        assert pol.state(k, rho, stag) == log_formula_bin(rho, k, stag)


def test_reward_hand_examples():
    for line in open(os.path.join(GOLD, "reward_hand_examples.txt")):
        if line.startswith("#") or not line.strip():
            continue
        cs, fs, fd, fa, rho, term, want = line.split()
        pol = O.OraclePolicy(cost=cs)
        a = 16 * int(fs) + 4 * int(fd) + int(fa)
        got = pol.reward(a, float(rho), int(term))
        assert abs(got - float(want)) < 1e-12


def test_log10_accuracy():
    rng = np.random.default_rng(1)
    xs = np.concatenate([10.0 ** rng.uniform(-300, 300, 5000), rng.uniform(0.5, 2.0, 2000),
                         [1.0, 10.0, 1e-8, 2.0 ** -1074, 1.7976931348623157e308]])
    for x in xs:
        got = O.log10(float(x))
        ref = math.log10(float(x))
        assert abs(got - ref) <= 4 * np.spacing(abs(ref)) + 1e-300
    assert math.isnan(O.log10(0.0)) and math.isnan(O.log10(-1.0))


def test_splitmix64_published_vector():
    want = [int(l) for l in open(os.path.join(GOLD, "splitmix64_seed1234567.txt"))
            if l.strip() and not l.startswith("#")]
    z = 1234567
    for w in want:
        assert O.mix64(z) == w
        z = (z + 0x9E3779B97F4A7C15) % 2 ** 64


def test_uniform_draws():
    us = np.array([O.uniform(7, 3, k, 0) for k in range(20000)])
    assert us.min() >= 0.0 and us.max() < 1.0
    assert abs(us.mean() - 0.5) < 0.01
    assert np.all(us * 2 ** 53 == np.floor(us * 2 ** 53))
    u1 = np.array([O.uniform(7, 3, k, 1) for k in range(2000)])
    assert not np.array_equal(us[:2000], u1)
    acts = np.floor(u1 * 64).astype(int)
    assert acts.min() == 0 and acts.max() == 63


def test_gelu_against_erf():
    for x in np.linspace(-8, 8, 4001):
        ref = 0.5 * x * (1 + math.erf(x / math.sqrt(2)))
        got = O.gelu(float(np.float32(x)))
        assert abs(got - ref) <= 3e-7 * abs(x) * 0.5 + 2e-6 * max(1.0, abs(x))


def eigvec_system():
    A = W.laplacian_2d(8)
    ev, V = np.linalg.eigh(A.to_dense())
    return A, V[:, 3].copy(), ev[3]


def test_q_update_terminal_one_step():
    """Eigenvector right-hand side: fp64 CG ends after one step, so one training
    episode makes one terminal update Q[s0,a] = lr * R (Algorithm 1, convergence branch)."""
    A, b, lam = eigvec_system()
    q0 = np.zeros((100, 64))
    q0[:, 63] = 1e-9                         # greedy picks fp64 everywhere
    pol = O.OraclePolicy(kind=O.POL_QTRAIN, q=q0, epsilon=0.0, cost="C1")
    x, info = O.cg(A, b, tol=1e-10, maxit=5, policy=pol, replace_period=50)
    assert info["status"] == 0 and info["iters"] == 1
    rho1 = info["rho"][1]
    s0 = pol.state(0, 1.0, 0)
    acc = 16.0 if rho1 <= 1e-16 else -math.log10(rho1)
    R = acc - 0.1 * 6.0 + 10.0
    assert abs(pol.q[s0, 63] - (1e-9 + 0.1 * (R - 1e-9))) < 1e-12
    changed = np.argwhere(pol.q != q0)
    assert changed.tolist() == [[s0, 63]]
    # repeated episodes move Q toward R geometrically: Q_e = R + (Q_0 - R)(1 - lr)^e
    for e in range(2, 6):
        O.cg(A, b, tol=1e-10, maxit=5, policy=pol, replace_period=50)
        assert abs(pol.q[s0, 63] - (R + (1e-9 - R) * 0.9 ** e)) < 1e-9


def test_q_update_bootstrapped_two_steps():
    """Two eigencomponents: two iterations.  The first transition bootstraps
    with gamma * max_a Q[s1, a] read before s1's own (terminal) update."""
    A = W.laplacian_2d(8)
    ev, V = np.linalg.eigh(A.to_dense())
    b = V[:, 2] + 0.5 * V[:, 40]
    q0 = np.zeros((100, 64))
    q0[:, 63] = 0.25
    pol = O.OraclePolicy(kind=O.POL_QTRAIN, q=q0, epsilon=0.0, cost="C2")
    x, info = O.cg(A, b, tol=1e-10, maxit=5, policy=pol, replace_period=50)
    assert info["status"] == 0 and info["iters"] == 2
    rho1, rho2 = info["rho"][1], info["rho"][2]
    s0 = pol.state(0, 1.0, 0)
    s1 = pol.state(1, rho1, 0)
    R0 = -math.log10(rho1) - 0.1 * 9.0
    R1 = (16.0 if rho2 <= 1e-16 else -math.log10(rho2)) - 0.1 * 9.0 + 10.0
    want0 = 0.25 + 0.1 * (R0 + 0.9 * 0.25 - 0.25)
    if s0 != s1:
        want1 = 0.25 + 0.1 * (R1 - 0.25)
        assert abs(pol.q[s0, 63] - want0) < 1e-12
    else:                                    # same cell: the terminal update follows the first
        want1 = want0 + 0.1 * (R1 - want0)
    assert abs(pol.q[s1, 63] - want1) < 1e-12
    assert np.count_nonzero(pol.q != q0) == len({s0, s1})


def test_epsilon_one_explores_with_counter_draws():
    A = W.laplacian_2d(16)
    b = W.rhs(A.n, 2)
    pol = O.OraclePolicy(kind=O.POL_QTRAIN, epsilon=1.0, seed=11, episode=4)
    x, info = O.cg(A, b, tol=1e-8, maxit=40, policy=pol, replace_period=50, fallback=True)
    k = info["iters"] if info["fallback_at"] < 0 else info["fallback_at"]
    acts = info["actions"][:k]
    want = [int(O.uniform(11, 4, i, 1) * 64) for i in range(k)]
    assert acts.tolist() == want
    assert np.all(info["flags"][:k] & O.FL_EXPLORED)


def mlp_weights(seed=0):
    rng = np.random.default_rng(seed)
    bf = lambda a: O.rd(a.astype(np.float32).astype(np.float64), O.BF16).astype(np.float32)
    return dict(W1=bf(rng.standard_normal((128, 16)) * 0.3), b1=rng.standard_normal(128).astype(np.float32) * 0.1,
                W2=bf(rng.standard_normal((128, 128)) * 0.1), b2=rng.standard_normal(128).astype(np.float32) * 0.1,
                W3=bf(rng.standard_normal((64, 128)) * 0.1), b3=rng.standard_normal(64).astype(np.float32) * 0.1)


def test_mlp_logits_against_float64_forward():
    torch = pytest.importorskip("torch")
    m = mlp_weights()
    pol = O.OraclePolicy(kind=O.POL_MLP, mlp=m)
    rng = np.random.default_rng(3)
    bf = lambda t: t.to(torch.bfloat16).to(torch.float64)
    g = lambda t: 0.5 * t * (1 + torch.erf(t / math.sqrt(2)))
    for _ in range(20):
        f = rng.standard_normal(16).astype(np.float32) * 3
        x = bf(torch.from_numpy(f).double())
        h1 = bf(g(torch.from_numpy(m["W1"]).double() @ x + torch.from_numpy(m["b1"]).double()))
        h2 = bf(g(torch.from_numpy(m["W2"]).double() @ h1 + torch.from_numpy(m["b2"]).double()))
        y = (torch.from_numpy(m["W3"]).double() @ h2 + torch.from_numpy(m["b3"]).double()).numpy()
        got = pol.mlp_logits(f)
        # bf16 rounding of h1/h2 can flip one ulp (2^-8 relative) between the two evaluations
        assert np.max(np.abs(got - y)) < 0.05 * (1 + np.max(np.abs(y)))
        assert np.corrcoef(got, y)[0, 1] > 0.999


def test_mlp_features():
    pol = O.OraclePolicy(kind=O.POL_MLP, mlp=mlp_weights(), replace_period=50)
    hist = np.array([1.0, 0.5, 0.1, 1e-3, 1e-4])
    f = pol.mlp_features(4, hist, 1, 2e-4, 16 * 1 + 4 * 2 + 3)
    lg = np.log10([1e-4, 1e-3, 0.1, 0.5, 1.0, 1.0, 1.0, 1.0])
    assert np.allclose(f[:8], lg, atol=1e-6)
    assert np.isclose(f[8], lg[0] - lg[1])
    assert np.isclose(f[9], 4 / 1000) and f[10] == 1.0
    assert np.isclose(f[11], math.log10(2e-4))
    assert np.isclose(f[12], 4 / 50)
    assert np.allclose(f[13:], [1 / 3, 2 / 3, 1.0])
