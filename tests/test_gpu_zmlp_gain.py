"""What the trained network gains over the method without it, on small systems.

The tabular Q-learning method of section 4.1 runs on small seeded systems and
its solves log (state, action, reward, next state) rollouts; the MLP policy is
trained on them by fitted Q-iteration on the matrix cores.  On held-out
systems of the same small family the trained network is then compared with
the Q-table it learned from (the method without the network), with the same
network untrained and with fp64 CG, every policy with the fp64 fallback.

The assertions fix what this seeded run shows: every policy reaches the
tolerance; against the Q-table the trained network has a lower abstract
precision cost, fewer fallbacks, fewer iterations and a shorter time; its
abstract cost is also below the untrained network's and fp64 CG's.  In time it
is slower than fp64 CG here (1.7x measured): at n <= 2e4 an iteration is bound
by launch latency, the same in every format, and the network's decision adds
one launch per iteration; the assertion bounds that overhead at 2.5x.

This gain does not carry over to the held-out systems of the large-scale
experiment (n up to 4M, kappa up to 1e8, a million rollouts; bench.py --mlp):
there the trained network falls back on every system and its median time is
about 2.2x fp64 CG's, behind the Q-table and the fixed mixed action."""
import json

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def family(seed):
    return W.family_system(seed, n_lo=2e3, n_hi=2e4, kappa_hi=1e5)


def test_trained_network_against_tabular_method():
    import torch

    import paper_2504_14268_amd as M

    systems = []
    for sd in range(500, 512):
        A = family(sd)
        m = M.Matrix(A)
        m.set_options(replace_period=50, fallback=True)
        systems.append((m, torch.from_numpy(W.rhs(A.n, sd)).cuda(), torch.empty(A.n, dtype=torch.float64, device="cuda")))
    P = M.Policy(kind=M.POLICY_QTABLE_TRAIN, cost="C1", seed=5)
    P.rollouts_enable(200000)
    M.train_qlearning(P, systems, episodes=4, maxit=600, order=1)
    roll = P.rollouts()
    n = len(roll["act"])
    assert n > 5000
    perm = np.random.default_rng(1).permutation(n)
    data = {k: torch.from_numpy(np.ascontiguousarray(v[perm])).cuda() for k, v in
            (("feat", roll["feat"]), ("next", roll["next"]), ("act", roll["act"].astype(np.int32)),
             ("rew", roll["rew"]), ("done", roll["done"]))}
    p0 = M.mlp_init_params(3)
    net = M.Mlp(p0)
    losses = net.train(data, batch=512, epochs=30, lr=1e-3, gamma=0.9)
    assert losses[-1] < losses[0]
    trained, untrained = M.Policy(kind=M.POLICY_MLP), M.Policy(kind=M.POLICY_MLP)
    net.to_policy(trained)
    M.Mlp(p0).to_policy(untrained)
    table = M.Policy(kind=M.POLICY_QTABLE, cost="C1")
    table.set_qtable(P.qtable())
    pols = {"fp64": M.Policy(kind=M.POLICY_FIXED, fixed_action=63), "qtable": table, "mlp_untrained": untrained,
            "mlp": trained}
    tot = {k: {"cost": 0.0, "iters": 0, "ms": 0.0, "fallbacks": 0, "ok": 0} for k in pols}
    held = range(600, 606)
    for sd in held:
        A = family(sd)
        m = M.Matrix(A)
        b = torch.from_numpy(W.rhs(A.n, sd)).cuda()
        x = torch.empty(A.n, dtype=torch.float64, device="cuda")
        for k, pol in pols.items():
            m.set_policy(pol)
            m.set_options(replace_period=50, fallback=True)
            x.zero_()
            r = m.solve(b, x, tol=1e-8, maxit=20000)
            t = tot[k]
            t["cost"] += r["cost_sum"]
            t["iters"] += r["iters"]
            t["ms"] += r["time_ms"]
            t["fallbacks"] += int(r["fallback_at"] >= 0)
            t["ok"] += int(r["status"] in (0, 2))
    ratios = {k: round(tot[k]["ms"] / tot["fp64"]["ms"], 3) for k in pols}
    per_it = {k: round(1e3 * tot[k]["ms"] / tot[k]["iters"], 2) for k in pols}
    print(json.dumps({"rollouts": n, "epoch_loss": [float(v) for v in losses], "heldout": tot,
                      "time_vs_fp64": ratios, "us_per_iteration": per_it}))
    for k in pols:
        assert tot[k]["ok"] == len(held), k
    # the gain over the tabular method: lower abstract cost, fewer fallbacks,
    # fewer iterations; and over the untrained network: lower cost
    assert tot["mlp"]["cost"] < tot["qtable"]["cost"]
    assert tot["mlp"]["fallbacks"] < tot["qtable"]["fallbacks"]
    assert tot["mlp"]["iters"] < tot["qtable"]["iters"]
    assert tot["mlp"]["cost"] < tot["mlp_untrained"]["cost"]
    assert tot["mlp"]["ms"] < tot["qtable"]["ms"]
    assert tot["mlp"]["ms"] < tot["mlp_untrained"]["ms"]
    # against fp64 CG: a lower abstract cost, and a time within the bound of
    # the per-iteration network decision on these launch-bound systems
    assert tot["mlp"]["cost"] < tot["fp64"]["cost"]
    assert tot["mlp"]["ms"] < 2.5 * tot["fp64"]["ms"]
