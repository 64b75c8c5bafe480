"""Benchmark: time to a true fp64 relative residual of 1e-8, mixed precision vs
fp64 CG, on one MI355X, plus the SpMV kernel's HBM bandwidth.

Workloads (synthetic, seeded):
  * 3D 7-point Laplacian 128^3 (n = 2,097,152, nnz = 14,581,760), b ~ U[-1,1]
    (seed 2), x0 = 0, tol 1e-8.  Mixed: SpMV in bf16 storage with fp32
    accumulation, dots and axpy in fp32, scalars in fp64, true residual
    recomputed in fp64 every 50 iterations.  fp64: plain fp64 CG.
  * random SPD, n = 1,000,000, 9..27 nnz/row, N(0,1) values, dominant diagonal,
    log-uniform diagonal scaling (matrix seed 3, b seed 4), same two solvers.
  Beside the headline: the single-reduction and pipelined variants of the
  iteration (two launches per iteration each) with the same actions, q52
  matrix storage, 16-bit vector storage, a learned Q-table
  and Jacobi preconditioning on the random SPD.

A step is one complete solve of the 3D Laplacian in mixed precision, inputs
resident in HBM.  `value` is its time to solution in ms (lower is better).
The SpMV roofline figure comes from HIP events around every SpMV launch of a
profiled solve, on the algorithmic bytes of one launch (each CSR entry once
with an int32 column index, the row pointers, p read once, q written once);
the bytes the kernel really streams (16-bit column deltas) are reported beside
it.  The CPU baseline is the oracle's plain fp64 CG on the host, run to
convergence on the same system, single-threaded, with an OpenMP variant on
every host core beside it.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time to true relres 1e-8 + SpMV HBM GB/s: mixed/learned vs fp64 CG, 1 GPU"
HBM_PEAK_GBS = 8000.0
COPY_BYTES = 256 << 20
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "spmv_traffic_lap3d_128.json")
KERNEL_SOURCES = ["paper_2504_14268_amd/csrc/kernels.hip", "paper_2504_14268_amd/csrc/dev.hpp",
                  "paper_2504_14268_amd/csrc/kernels.hpp"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def ka_bytes(n: int, nnz: int, fs: int, vec_bytes: int, idx_bytes: int = 4) -> int:
    """Algorithmic bytes of one iteration launch of KA (SpMV q = A p with the
    p.q partial): each CSR entry once (value + column index: int32, or the
    16-bit delta col - row where the matrix has them), the row pointers, p read
    once and q written once; fp16 adds the one-byte row exponents."""
    val = {0: 2, 1: 2, 2: 4, 3: 8, 4: 1}[fs]
    b = nnz * (val + idx_bytes) + 4 * (n + 1) + 2 * n * vec_bytes
    if fs in (0, 4):       # fp16 and q52 read the row exponents
        b += n
    return b


def cpu_model() -> str:
    """The host CPU's model name (Linux /proc/cpuinfo), or "unknown"."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def mix_of(M, actions) -> dict:
    """Share of each format per operation over a solve's actions."""
    a = np.asarray(actions, dtype=np.int64)
    if a.size == 0:
        return {}
    names = ("fp16", "bf16", "fp32", "fp64", "q52", "tf32")
    fm = formats_of(M, a)
    out = {}
    for j, op in enumerate(("spmv", "dot", "axpy")):
        f = fm[:, j]
        out[op] = {names[i]: round(float(np.mean(f == i)), 3) for i in range(6) if np.any(f == i)}
    return out


def formats_of(M, actions) -> np.ndarray:
    """[len, 3] format codes (spmv, dot, axpy) of action codes, by the library's decoding."""
    a = np.asarray(actions, dtype=np.int64)
    u, inv = np.unique(a, return_inverse=True)
    table = np.array([M.decode(int(v)) for v in u], dtype=np.int64).reshape(-1, 3)
    return table[inv.reshape(-1)]


def build_systems(M, W, torch, seeds, n_hi=5e5, kappa_hi=1e8):
    """Device systems (Matrix, b, x) of family_system(seed), b ~ U[-1,1] (seed + 10000)."""
    systems = []
    for sd in seeds:
        A = W.family_system(sd, n_hi=n_hi, kappa_hi=kappa_hi)
        mm = M.Matrix(A)
        mm.set_options(replace_period=50, fallback=True)
        b = torch.from_numpy(W.rhs(A.n, sd + 10000)).cuda()
        systems.append((mm, b, torch.empty(A.n, dtype=torch.float64, device="cuda")))
    return systems


# Cost per format measured on this GPU (a labelled variation of the cost
# settings C1 / C2): the fp64 kernels of an iteration take 1.8-1.9x the fp32
# ones (SpMV 35.6 vs 19.4 us, axpy+dot 22.2 vs 11.5 us, direction 12.1 vs
# 6.8 us on the 3D Laplacian 128^3), and fp16 / bf16 dots and updates run in
# fp32 containers, at fp32's time.
COST_HW = (1.0, 1.0, 1.0, 1.9)


def cost_table(name):
    return COST_HW if name == "Chw" else name


def train_qtable(M, systems, episodes, maxit, cost, seed=12345, rollouts=0, w1=1.0, gamma=0.9, D=1, per_op=0):
    """Trains a device Q-table (Algorithm 1) over the systems, episode sweeps.
    w1: weight of the reward's accuracy term (section 4.1: 1.0); gamma: the
    discount (section 5: 0.9); D: the decision period (1: every iteration);
    per_op: one Q-table per operation (section 4.1) instead of a joint one."""
    P = M.Policy(kind=M.POLICY_QTABLE_TRAIN, cost=cost_table(cost), seed=seed, w=(w1, 0.1, 10.0), gamma=gamma,
                 decision_period=D, per_op=per_op)
    if rollouts:
        P.rollouts_enable(rollouts)
    res = M.train_qlearning(P, systems, episodes=episodes, maxit=maxit, tol=1e-8, eps_start=1.0,
                            eps_end=0.1, order=1)
    return P, res


def iteration_bytes(n: int, nnz: int, fs: int, vb: int) -> int:
    """Algorithmic bytes of one CG iteration: SpMV (values, indices, row
    pointers, p in, q out), axpy + dot (6 vectors), direction update (3)."""
    val = {0: 2, 1: 2, 2: 4, 3: 8}[fs]
    return nnz * (val + 4) + 4 * (n + 1) + 11 * n * vb + (n if fs == 0 else 0)


def batched_experiment(args, M, W, torch) -> dict:
    """Batched solve of uneven SPD systems (banded and random pattern, n
    log-uniform in [1e3, 2e5], cond log-uniform in [1e2, 1e4]): one persistent
    launch (autotuned) against one mpcg_solve per system, bf16 SpMV with fp32
    dots and axpy, and the same batch in fp64."""
    seeds = range(1000, 1000 + args.batch_systems)
    t0 = time.time()
    mats, bs, xs, shapes = [], [], [], []
    act = M.action(M.BF16, M.FP32, M.FP32)
    pol = M.Policy(kind=M.POLICY_FIXED, fixed_action=act)
    pol64 = M.Policy(kind=M.POLICY_FIXED, fixed_action=63)
    for sd in seeds:
        A = W.batch_system(sd)
        m = M.Matrix(A)
        m.set_policy(pol)
        m.set_options(replace_period=50, fallback=True)
        mats.append(m)
        bs.append(torch.from_numpy(W.rhs(A.n, sd + 5000)).cuda())
        xs.append(torch.zeros(A.n, dtype=torch.float64, device="cuda"))
        shapes.append((A.n, A.nnz))
        del A
    setup_s = time.time() - t0
    sum_n = sum(n for n, _ in shapes)
    sum_nnz = sum(z for _, z in shapes)
    log(f"[batched] {len(mats)} systems, sum n {sum_n}, sum nnz {sum_nnz}, built in {setup_s:.1f} s")
    systems = list(zip(mats, bs, xs))
    maxit = 20000

    def zero():
        for x in xs:
            x.zero_()

    zero()
    res_t, info_t = M.solve_batched(systems, tol=1e-8, maxit=maxit)        # autotunes, then solves
    log(f"[batched] autotuned: {info_t}")
    assert all(r["status"] in (0, 2) for r in res_t), "a batched system did not converge"
    runs = []
    for _ in range(2):
        zero()
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        res_b, info_b = M.solve_batched(systems, tol=1e-8, maxit=maxit)
        runs.append((time.perf_counter() - w0, res_b, info_b))
    wall_b, res_b, info_b = min(runs, key=lambda r: r[0])
    xb = [x.clone() for x in xs]
    log(f"[batched] one launch: {info_b['time_ms']:.1f} ms device, {wall_b * 1e3:.1f} ms wall")
    # one solve per system, same stream order
    zero()
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    res_s = [m.solve(b, x, tol=1e-8, maxit=maxit) for m, b, x in systems]
    torch.cuda.synchronize()
    wall_s = time.perf_counter() - w0
    same = all(r1["status"] == r2["status"] and r1["iters"] == r2["iters"] for r1, r2 in zip(res_b, res_s)) and \
        all(torch.equal(a, b) for a, b in zip(xb, xs))
    log(f"[batched] sequential: {wall_s * 1e3:.1f} ms wall; identical results: {same}")
    for m in mats:
        m.set_policy(pol64)
    zero()
    res_64, info_64 = M.solve_batched(systems, tol=1e-8, maxit=maxit)
    it = np.array([r["iters"] for r in res_b])
    alg = sum(r["iters"] * iteration_bytes(n, z, M.BF16, 4) for r, (n, z) in zip(res_b, shapes))
    alg64 = sum(r["iters"] * iteration_bytes(n, z, M.FP64, 8) for r, (n, z) in zip(res_64, shapes))
    out = {"experiment": "batched persistent solve", "systems": len(mats), "sum_n": sum_n, "sum_nnz": sum_nnz,
           "setup_s": round(setup_s, 1), "action": "bf16 SpMV, fp32 dot, fp32 axpy, R=50, fp64 fallback on stagnation",
           "config": {k: info_b[k] for k in ("strategy", "workgroups", "spmv_rows", "split_rows", "n_split")},
           "persistent_ms": round(info_b["persistent_ms"], 2), "split_ms": round(info_b["split_ms"], 2),
           "fallbacks": int(sum(1 for r in res_b if r["fallback_at"] >= 0)),
           "autotune_ms": round(info_t["tune_ms"], 1),
           "batched_ms": round(info_b["time_ms"], 2), "batched_wall_ms": round(wall_b * 1e3, 2),
           "sequential_wall_ms": round(wall_s * 1e3, 2),
           "speedup_vs_sequential": round(wall_s / wall_b, 2),
           "batched_fp64_ms": round(info_64["time_ms"], 2),
           "speedup_vs_batched_fp64": round(info_64["time_ms"] / info_b["time_ms"], 3),
           "identical_to_sequential": bool(same),
           "converged": int(sum(1 for r in res_b if r["status"] == 0)),
           "iterations": {"min": int(it.min()), "median": int(np.median(it)), "max": int(it.max()), "sum": int(it.sum())},
           "aggregate_GBps": round(alg / (info_b["time_ms"] * 1e-3) / 1e9, 1),
           "aggregate_GBps_fp64": round(alg64 / (info_64["time_ms"] * 1e-3) / 1e9, 1)}
    for m in mats:
        m.close()
    return out


MLP_FLOPS_PER_SAMPLE_EPOCH = 2 * (16 * 128 + 128 * 128 + 128 * 64) * 2 + 2 * (128 * 64 + 128 * 128 + 16 * 128 +
                                                                             128 * 128 + 128 * 64)


def evaluate_policies(M, W, torch, seeds, policies: dict, maxit: int, family=None) -> tuple:
    """Solves each held-out system with every policy (fallback on); per-system rows and a summary."""
    family = family or W.family_system
    rows = []
    for sd in seeds:
        A = family(sd)
        mm = M.Matrix(A)
        b = torch.from_numpy(W.rhs(A.n, sd + 10000)).cuda()
        x = torch.empty(A.n, dtype=torch.float64, device="cuda")
        row = {"seed": sd, "name": A.name, "n": A.n, "nnz": A.nnz}
        for lab, pol in policies.items():
            mm.set_policy(pol)
            mm.set_options(replace_period=50, fallback=True, profile=False)
            x.zero_()
            r = mm.solve(b, x, tol=1e-8, maxit=maxit)
            if A.n >= 1_000_000:
                log(f"[eval] {sd} {A.name} {lab}: {r['status']}/{r['iters']}/{r['time_ms']:.1f}ms")
            row[lab] = {"status": r["status"], "iters": r["iters"], "ms": round(r["time_ms"], 3),
                        "relres_true": r["relres_true"], "cost_sum": r["cost_sum"], "fallback_at": r["fallback_at"]}
            if lab not in ("fp64",):
                row[lab]["mix"] = mix_of(M, mm.history()["actions"])
        rows.append(row)
        log(f"[eval] {sd} {A.name}: " + ", ".join(f"{k} {row[k]['status']}/{row[k]['iters']}/{row[k]['ms']}ms"
                                                   for k in policies))
        mm.close()
    summ = {}
    for lab in policies:
        ok = [r for r in rows if r[lab]["status"] in (0, 2)]
        both = [r for r in ok if r["fp64"]["status"] in (0, 2)] if "fp64" in policies else []
        summ[lab] = {"success": f"{len(ok)}/{len(rows)}",
                     "fallbacks": sum(1 for r in rows if r[lab]["fallback_at"] >= 0),
                     "total_ms": round(sum(r[lab]["ms"] for r in rows), 1),
                     "total_iters": int(sum(r[lab]["iters"] for r in rows)),
                     "total_cost": round(sum(r[lab]["cost_sum"] for r in rows), 1),
                     "median_time_ratio_vs_fp64": round(float(np.median([r[lab]["ms"] / r["fp64"]["ms"] for r in both])), 3)
                     if both else None}
    return rows, summ


def mlp_experiment(args, M, W, torch) -> dict:
    """Learned MLP policy: rollouts logged by the solver during tabular Q-learning
    (section 4.1) on seeded training systems, the network trained on them by
    fitted Q-iteration on the matrix cores, then compared on held-out systems
    with the Q-table it came from, the untrained network, fixed mixed precision
    and fp64 CG (every policy with the fp64 fallback)."""
    out = {"experiment": "MLP precision policy"}
    t0 = time.time()
    systems = build_systems(M, W, torch, range(100, 100 + args.train_systems))
    out["train_systems"] = len(systems)
    log(f"[mlp] {len(systems)} training systems built in {time.time() - t0:.1f} s")
    t0 = time.time()
    P, res = train_qtable(M, systems, args.episodes, 1000, "C1", rollouts=1_000_000, w1=args.w1)
    roll = P.rollouts()
    n = len(roll["act"])
    out["qlearning"] = {"episodes": len(res), "wall_s": round(time.time() - t0, 1), "rollouts": n,
                        "reward_weights": [args.w1, 0.1, 10.0]}
    log(f"[mlp] Q-learning: {out['qlearning']}")
    for mm, _, _ in systems:
        mm.close()
    del systems
    perm = np.random.default_rng(2024).permutation(n)
    data = {"feat": roll["feat"][perm], "next": roll["next"][perm], "act": roll["act"][perm].astype(np.int32),
            "rew": roll["rew"][perm].astype(np.float32), "done": roll["done"][perm].astype(np.uint8)}
    dd = {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in data.items()}
    p0 = M.mlp_init_params(77)
    net = M.Mlp(p0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = net.train(dd, batch=512, epochs=args.mlp_epochs, lr=1e-3, gamma=0.9)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    used = (n // 512) * 512
    flops = MLP_FLOPS_PER_SAMPLE_EPOCH * used * args.mlp_epochs
    out["training"] = {"samples": used, "epochs": args.mlp_epochs, "batch": 512, "wall_s": round(dt, 3),
                       "samples_per_s": round(used * args.mlp_epochs / dt, 0),
                       "TFLOPs": round(flops / dt / 1e12, 3), "bf16_peak_TFLOPs": 2500.0,
                       "epoch_loss": [round(float(l), 5) for l in losses]}
    log(f"[mlp] training: {out['training']}")
    mlp_pol = M.Policy(kind=M.POLICY_MLP)
    net.to_policy(mlp_pol)
    untrained = M.Policy(kind=M.POLICY_MLP)
    M.Mlp(p0).to_policy(untrained)
    greedy = M.Policy(kind=M.POLICY_QTABLE, cost="C1")
    greedy.set_qtable(P.qtable())
    pols = {"fp64": M.Policy(kind=M.POLICY_FIXED, fixed_action=63),
            "fixed_mixed": M.Policy(kind=M.POLICY_FIXED, fixed_action=M.action(M.BF16, M.FP32, M.FP32)),
            "qtable": greedy, "mlp_untrained": untrained, "mlp": mlp_pol}
    if args.spmv_only:
        # labelled variation: the learned choice restricted to the SpMV format,
        # dots and updates in fp32 (the other actions masked: -2^100 on the
        # network's output bias, -1e300 in the table)
        keep = [M.action(fs, M.FP32, M.FP32) for fs in (M.FP16, M.BF16, M.FP32, M.FP64)]
        masked = np.ones(64, dtype=bool)
        masked[keep] = False
        pm = net.params()
        pm["b3"] = pm["b3"].copy()
        pm["b3"][masked] = np.float32(-2.0 ** 100)
        mlp_sp = M.Policy(kind=M.POLICY_MLP)
        M.Mlp(pm).to_policy(mlp_sp)
        q = P.qtable().copy()
        q[:, masked] = -1e300
        q_sp = M.Policy(kind=M.POLICY_QTABLE, cost="C1")
        q_sp.set_qtable(q)
        pols["qtable_spmv_only"] = q_sp
        pols["mlp_spmv_only"] = mlp_sp
    s0 = args.heldout_seed0
    out["heldout"] = {"seeds": [s0, s0 + args.heldout_systems - 1], "n_hi": args.heldout_n_hi,
                      "maxit": args.eval_maxit}
    rows, summ = evaluate_policies(M, W, torch, range(s0, s0 + args.heldout_systems), pols, args.eval_maxit,
                                   family=lambda sd: W.family_system(sd, n_hi=args.heldout_n_hi))
    out["heldout_summary"] = summ
    out["heldout_rows"] = rows
    return out


def paper_experiment(args, M, W, torch) -> dict:
    """Section 5's setting on its two synthetic families: one Q-table per
    operation (section 4.1) over fp16, bf16, tf32, fp32 and fp64, cost
    settings C1 and C2, 10
    training matrices x 200 episodes, epsilon 1 -> 0.1, the termination
    rho < 1e-6 with k >= 10 and T_max = 1000, no periodic residual replacement;
    then 100 test matrices against fp64 CG: iterations, the relative error
    against a direct solve, and the share of each format per operation (the
    analogues of Tables 2-4; the paper's matrices and seeds are not published,
    so the comparison is qualitative).  Both readings of a low-precision
    operation are run: the paper's emulation (an fp64 operation whose result is
    rounded) and the hardware one (formats in memory and arithmetic)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spl

    families = {
        "bbt_5000": lambda sd: (lambda A: (A, W.rhs(A.n, sd + 7)))(W.bbt_system(sd, density_reading="pairs")),
        "poisson_80": lambda sd: W.poisson_subdomain(sd),
    }
    tol, T = 1e-6, 1000
    out = {"experiment": "paper setting (section 5)", "tol": tol, "T_max": T, "k_min": 10,
           "train_matrices": args.paper_train, "episodes_per_matrix": args.paper_episodes,
           "test_matrices": args.paper_test, "per_op": args.paper_per_op, "rho_fp64": args.paper_rho64,
           "formats": ["fp16", "bf16", "fp32", "fp64"] + (["tf32"] if args.paper_nfmt == 5 else [])}
    names = ("fp16", "bf16", "fp32", "fp64", "q52", "tf32")
    for reading in args.paper_readings.split(","):
        emu = {"emulation": 1, "hardware": 0}[reading]
        out[reading] = {}
        for fam, gen in families.items():
            t0 = time.time()
            train = []
            for sd in range(3000, 3000 + args.paper_train):
                A, b = gen(sd)
                mm = M.Matrix(A)
                mm.set_options(replace_period=0, fallback=False, stop_rule=1, rho_fp64=args.paper_rho64,
                               emulate=emu)
                train.append((mm, torch.from_numpy(np.ascontiguousarray(b)).cuda(),
                              torch.empty(A.n, dtype=torch.float64, device="cuda")))
            tables = {}
            fo = {"train_setup_s": round(time.time() - t0, 1)}
            for cost in ("C1", "C2"):
                P = M.Policy(kind=M.POLICY_QTABLE_TRAIN, cost=cost, seed=31, per_op=args.paper_per_op,
                             nfmt=args.paper_nfmt)
                t0 = time.time()
                res = M.train_qlearning(P, train, episodes=args.paper_episodes, maxit=T, tol=tol, eps_start=1.0,
                                        eps_end=0.1, order=1)
                fo[f"train_{cost}_s"] = round(time.time() - t0, 1)
                fo[f"train_{cost}_converged_share"] = round(float(np.mean([r["status"] == 0 for r in res])), 3)
                g = M.Policy(kind=M.POLICY_QTABLE, cost=cost, per_op=args.paper_per_op, nfmt=args.paper_nfmt)
                g.set_qtable(P.qtable())
                tables[cost] = g
                log(f"[paper] {reading} {fam} {cost}: trained {len(res)} episodes in {fo[f'train_{cost}_s']} s")
            for mm, _, _ in train:
                mm.close()
            # the fixed legs isolate the storage format of A: SpMV at fp16, bf16 or
            # fp32, everything else in fp64
            pols = {"fp64": M.Policy(kind=M.POLICY_FIXED, fixed_action=63),
                    "spmv_fp16_rest_fp64": M.Policy(kind=M.POLICY_FIXED, fixed_action=M.action(M.FP16, M.FP64, M.FP64)),
                    "spmv_bf16_rest_fp64": M.Policy(kind=M.POLICY_FIXED, fixed_action=M.action(M.BF16, M.FP64, M.FP64)),
                    "spmv_fp32_rest_fp64": M.Policy(kind=M.POLICY_FIXED, fixed_action=M.action(M.FP32, M.FP64, M.FP64)),
                    "RL_C1": tables["C1"], "RL_C2": tables["C2"]}
            stats = {k: {"iters": [], "err": [], "ms": [], "status": [], "mix": np.zeros((3, 6))} for k in pols}
            for sd in range(4000, 4000 + args.paper_test):
                A, b = gen(sd)
                S = sp.csr_matrix((A.val, A.col, A.row_ptr), shape=(A.n, A.n))
                x_ref = spl.spsolve(S.tocsc(), b)
                mm = M.Matrix(A)
                bd = torch.from_numpy(np.ascontiguousarray(b)).cuda()
                xd = torch.empty(A.n, dtype=torch.float64, device="cuda")
                for k, pol in pols.items():
                    mm.set_policy(pol)
                    mm.set_options(replace_period=0, fallback=False, stop_rule=1, rho_fp64=args.paper_rho64,
                               emulate=emu)
                    xd.zero_()
                    r = mm.solve(bd, xd, tol=tol, maxit=T)
                    x = xd.cpu().numpy()
                    st = stats[k]
                    st["iters"].append(r["iters"])
                    st["status"].append(r["status"])
                    st["ms"].append(r["time_ms"])
                    st["err"].append(float(np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref)))
                    fm = formats_of(M, mm.history()["actions"][:r["iters"]])
                    for j in range(3):
                        st["mix"][j] += np.bincount(fm[:, j], minlength=6)[:6]
                mm.close()
            fo["test"] = {}
            for k, st in stats.items():
                it, er, stt = np.array(st["iters"]), np.array(st["err"]), np.array(st["status"])
                mix = st["mix"] / np.maximum(st["mix"].sum(axis=1, keepdims=True), 1)
                fo["test"][k] = {"mean_iters": round(float(it.mean()), 1), "std_iters": round(float(it.std()), 1),
                                 "p75_iters": float(np.percentile(it, 75)),
                                 "status_counts": {int(v): int(np.sum(stt == v)) for v in np.unique(stt)},
                                 "mean_rel_error": float(er.mean()), "max_rel_error": float(er.max()),
                                 "median_rel_error": float(np.median(er)),
                                 "p25_p75_rel_error": [float(np.percentile(er, 25)), float(np.percentile(er, 75))],
                                 "total_ms": round(float(np.sum(st["ms"])), 2),
                                 "mix": {op: {names[f]: round(float(mix[j, f]), 3) for f in range(6) if f != 4}
                                         for j, op in enumerate(("spmv", "dot", "update"))}}
            log(f"[paper] {reading} {fam}: " + json.dumps({k: (v["mean_iters"], v["mean_rel_error"]) for k, v in fo["test"].items()}))
            out[reading][fam] = fo
    return out


def qlearning_experiment(args, M, W, torch) -> dict:
    """Tabular Q-learning on seeded systems (2D/3D Laplacians and random SPD,
    n log-uniform in [1e4, 5e5], cond up to 1e8), then greedy inference on
    held-out seeds against the fixed mixed action and fp64 CG."""
    train_seeds = range(100, 100 + args.train_systems)
    held = range(300, 300 + args.heldout_systems)
    out = {"experiment": "tabular Q-learning precision policy", "train_seeds": [train_seeds[0], train_seeds[-1]],
           "heldout_seeds": [held[0], held[-1]], "episodes_per_system": args.episodes,
           "train_maxit": 1000, "eval_maxit": args.eval_maxit}
    policies = {}
    t0 = time.time()
    systems = build_systems(M, W, torch, train_seeds)
    out["train_setup_s"] = round(time.time() - t0, 1)
    log(f"[qlearning] {len(systems)} training systems built in {out['train_setup_s']} s")
    if args.variants:
        variants = []
        for v in args.variants.split(","):
            f = v.split(":") + ["1.0", "0.9", "1", "0"][len(v.split(":")) - 1:]
            variants.append((f[0], float(f[1]), float(f[2]), int(f[3]), int(f[4])))
    else:
        variants = [("C1", 1.0, 0.9, 1, 0), ("C2", 1.0, 0.9, 1, 0)] + (
            [("C1", 0.0, 0.9, 1, 0), ("C2", 0.0, 0.9, 1, 0)] if args.w1_variation else [])
    for cost, w1, gamma, D, per_op in variants:
        lab = (cost + ("" if w1 == 1.0 else f"_w1_{w1:g}") + ("" if gamma == 0.9 else f"_g{gamma:g}")
               + ("" if D == 1 else f"_D{D}") + ("" if not per_op else "_perop" if per_op == 1 else "_perop2"))
        t0 = time.time()
        P, res = train_qtable(M, systems, args.episodes, 1000, cost, w1=w1, gamma=gamma, D=D, per_op=per_op)
        dt = time.time() - t0
        it = np.array([r["iters"] for r in res])
        conv = np.array([r["status"] in (0, 2) for r in res])
        sweeps = np.array_split(np.arange(len(res)), args.episodes)
        out[f"train_{lab}"] = {"wall_s": round(dt, 1), "episodes": len(res), "w1": w1, "gamma": gamma, "D": D,
                               "per_op": per_op,
                               "cost_table": list(cost_table(cost)) if cost == "Chw" else cost,
                                "iterations": int(it.sum()),
                                "converged_share_per_sweep": [round(float(conv[s].mean()), 3) for s in sweeps],
                                "mean_cost_per_iteration_per_sweep": [
                                    round(float(sum(res[j]["cost_sum"] for j in s) / max(1, sum(res[j]["iters"] for j in s))), 3)
                                    for s in sweeps]}
        log(f"[qlearning] {lab}: {out[f'train_{lab}']}")
        policies[lab] = (P, cost, D, per_op)
    for mm, _, _ in systems:
        mm.close()
    del systems
    fixed = M.Policy(kind=M.POLICY_FIXED, fixed_action=M.action(M.BF16, M.FP32, M.FP32))
    fp64 = M.Policy(kind=M.POLICY_FIXED, fixed_action=63)
    greedy = {}
    for lab, (P, cost, D, per_op) in policies.items():
        g = M.Policy(kind=M.POLICY_QTABLE, cost=cost_table(cost), decision_period=D, per_op=per_op)
        g.set_qtable(P.qtable())
        greedy[lab] = g
        if args.spmv_only and per_op in (0, 1):
            q = P.qtable().copy()
            if per_op == 1:
                # the learned SpMV table; the dot and update tables masked so
                # that their greedy choice is fp32 (columns 4 + d and 8 + d)
                for j in (1, 2):
                    for d in range(4):
                        if d != M.FP32:
                            q[:, 4 * j + d] = -1e300
            else:
                # the joint table restricted to the four (f_s, fp32, fp32) actions
                keep = [M.action(fs, M.FP32, M.FP32) for fs in (M.FP16, M.BF16, M.FP32, M.FP64)]
                q[:, [a for a in range(64) if a not in keep]] = -1e300
            gm = M.Policy(kind=M.POLICY_QTABLE, cost=cost_table(cost), decision_period=D, per_op=per_op)
            gm.set_qtable(q)
            greedy[lab + "_spmv_only"] = gm
    labels = ["fp64", "fixed_mixed"] + [f"learned_{lab}" for lab in greedy]
    rows = []
    for sd in held:
        A = W.family_system(sd)
        mm = M.Matrix(A)
        b = torch.from_numpy(W.rhs(A.n, sd + 10000)).cuda()
        x = torch.empty(A.n, dtype=torch.float64, device="cuda")
        row = {"seed": sd, "name": A.name, "n": A.n, "nnz": A.nnz}
        for lab, pol in [("fp64", fp64), ("fixed_mixed", fixed)] + [(f"learned_{k}", g) for k, g in greedy.items()]:
            mm.set_policy(pol)
            mm.set_options(replace_period=50, fallback=True)
            x.zero_()
            r = mm.solve(b, x, tol=1e-8, maxit=args.eval_maxit)
            row[lab] = {"status": r["status"], "iters": r["iters"], "ms": round(r["time_ms"], 3),
                        "relres_true": r["relres_true"], "cost_sum": r["cost_sum"],
                        "fallback_at": r["fallback_at"]}
            if lab.startswith("learned"):
                row[lab]["mix"] = mix_of(M, mm.history()["actions"])
        rows.append(row)
        log(f"[qlearning] held-out {sd} {A.name}: " +
            ", ".join(f"{k} {row[k]['status']}/{row[k]['iters']}/{row[k]['ms']}ms" for k in labels))
        mm.close()
    summ = {}
    for lab in labels:
        ok = [r for r in rows if r[lab]["status"] in (0, 2)]
        both = [r for r in rows if r[lab]["status"] in (0, 2) and r["fp64"]["status"] in (0, 2)]
        summ[lab] = {"success": f"{len(ok)}/{len(rows)}",
                     "fallbacks": sum(1 for r in rows if r[lab]["fallback_at"] >= 0),
                     "median_time_ratio_vs_fp64": round(float(np.median([r[lab]["ms"] / r["fp64"]["ms"] for r in both])), 3)
                     if both else None,
                     "median_iter_ratio_vs_fp64": round(float(np.median([r[lab]["iters"] / r["fp64"]["iters"] for r in both])), 3)
                     if both else None,
                     "total_ms": round(sum(r[lab]["ms"] for r in rows), 1)}
    out["heldout_summary"] = summ
    out["heldout"] = rows
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-rspd", action="store_true", help="skip the random SPD workload")
    ap.add_argument("--N", type=int, default=128, help="3D Laplacian grid size")
    ap.add_argument("--qlearning", action="store_true",
                    help="tabular Q-learning experiment: train on seeded systems, evaluate on held-out ones")
    ap.add_argument("--train-systems", type=int, default=200)
    ap.add_argument("--heldout-systems", type=int, default=50)
    ap.add_argument("--episodes", type=int, default=5)
    ap.add_argument("--eval-maxit", type=int, default=20000)
    ap.add_argument("--w1-variation", action="store_true",
                    help="also train with the reward's accuracy weight w1 = 0 (a labelled variation; "
                         "section 4.1's weights are (1, 0.1, 10))")
    ap.add_argument("--w1", type=float, default=1.0, help="accuracy weight of the MLP experiment's reward")
    ap.add_argument("--variants", default="",
                    help="Q-learning variants cost[:w1[:gamma[:D[:per_op]]]], comma separated (cost C1, C2 "
                         "or Chw, the cost per format measured on this GPU; D the decision period; per_op 1 for "
                         "one Q-table per operation); default: C1 and C2 with section 4.1's weights, a joint "
                         "table, decisions every iteration")
    ap.add_argument("--spmv-only", action="store_true",
                    help="also evaluate the learned policies restricted to the SpMV format, dots and updates "
                         "masked to fp32 (a labelled variation; the joint and per-operation tables in "
                         "--qlearning, the joint table and the network in --mlp)")
    ap.add_argument("--heldout-n-hi", type=float, default=5e5, help="largest held-out system size")
    ap.add_argument("--heldout-seed0", type=int, default=2000, help="first held-out seed of the MLP experiment")
    ap.add_argument("--paper", action="store_true",
                    help="section 5's setting on its synthetic families (per-operation Q-tables, rho < 1e-6 "
                         "with k >= 10, T_max 1000) against fp64 CG")
    ap.add_argument("--paper-train", type=int, default=10)
    ap.add_argument("--paper-episodes", type=int, default=200)
    ap.add_argument("--paper-per-op", type=int, default=2, choices=(1, 2),
                    help="1: a table per operation for SpMV, dot and updates; 2: SpMV and dot, updates in fp64")
    ap.add_argument("--paper-test", type=int, default=100)
    ap.add_argument("--paper-readings", default="emulation,hardware",
                    help="emulation: the paper's reading (fp64 operations, results rounded to each "
                         "operation's format); hardware: this library's formats in memory and arithmetic")
    ap.add_argument("--paper-nfmt", type=int, default=5, choices=(4, 5),
                    help="5: the paper's format set with tf32 (emulated), 4: without it")
    ap.add_argument("--paper-rho64", type=int, default=1, choices=(0, 1),
                    help="1: rho from an fp64 r.r (the paper keeps residual computations in fp64)")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-policy leg")
    ap.add_argument("--batched", action="store_true",
                    help="batched experiment: 512 uneven systems in one persistent launch vs sequential solves")
    ap.add_argument("--batch-systems", type=int, default=512)
    ap.add_argument("--mlp", action="store_true",
                    help="MLP policy experiment: rollouts from Q-learning runs, matrix-core training, held-out comparison")
    ap.add_argument("--mlp-epochs", type=int, default=30)
    ap.add_argument("--counters", action="store_true",
                    help="short run for HBM counter collection: one plain copy of 256 MiB (the scale "
                         "reference for FETCH_SIZE / WRITE_SIZE), then one mixed solve")
    ap.add_argument("--counters-system", choices=["lap3d", "rspd"], default="lap3d",
                    help="system of the counter run: the 3D Laplacian or the random SPD (n = 1e6)")
    ap.add_argument("--counters-maxit", type=int, default=5000,
                    help="iteration budget of the counter run's solve")
    ap.add_argument("--counters-fp64", action="store_true", help="counter run with the fp64 action")
    ap.add_argument("--counters-variant", type=int, choices=[0, 1, 2], default=0,
                    help="counter run with the single-reduction (1) or pipelined (2) CG")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the solver runs on one GPU only (--gpus {args.gpus} requested); "
              "a multi-GPU row decomposition is not implemented.", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2504_14268_amd as M
    import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    dev_name = torch.cuda.get_device_name(0)
    tol = 1e-8
    act_mixed = M.action(M.BF16, M.FP32, M.FP32)
    act_fp64 = M.action(M.FP64, M.FP64, M.FP64)

    t0 = time.time()
    A = W.laplacian_3d(args.N)
    b = W.rhs(A.n, 2)
    log(f"[bench] generated {A.name} n={A.n} nnz={A.nnz} in {time.time() - t0:.1f}s")
    t0 = time.time()
    m = M.Matrix(A)
    torch.cuda.synchronize()
    setup_ms = (time.time() - t0) * 1e3
    bd = torch.from_numpy(b).cuda()
    xd = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    pol_mixed = M.Policy(kind=M.POLICY_FIXED, fixed_action=act_mixed)
    pol_fp64 = M.Policy(kind=M.POLICY_FIXED, fixed_action=act_fp64)

    if args.mlp:
        print(json.dumps(mlp_experiment(args, M, W, torch)), flush=True)
        return

    if args.batched:
        print(json.dumps(batched_experiment(args, M, W, torch)), flush=True)
        return

    if args.qlearning:
        print(json.dumps(qlearning_experiment(args, M, W, torch)), flush=True)
        return

    if args.paper:
        print(json.dumps(paper_experiment(args, M, W, torch)), flush=True)
        return

    if args.counters:
        if args.counters_system == "rspd":
            A = W.random_spd(1_000_000, 3, W.spread_for_kappa(1e6))
            m = M.Matrix(A)
            bd = torch.from_numpy(W.rhs(A.n, 4)).cuda()
            xd = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        pol = pol_fp64 if args.counters_fp64 else pol_mixed
        fs, vb = (M.FP64, 8) if args.counters_fp64 else (M.BF16, 4)
        m.set_policy(pol)
        R = 0 if args.counters_fp64 else 20 if args.counters_variant == 2 else 50
        m.set_options(replace_period=R, fallback=False, variant=args.counters_variant)
        r = m.solve(bd, xd, tol=tol, maxit=args.counters_maxit)
        print(json.dumps({"counters_run": True, "system": A.name, "n": A.n, "nnz": A.nnz,
                          "action": "fp64" if args.counters_fp64 else "mixed", "variant": args.counters_variant,
                          "copy_bytes": COPY_BYTES,
                          "iters": r["iters"], "relres_true": r["relres_true"], "kernel_hash": kernel_hash(),
                          "algorithmic_bytes_per_launch_ka": ka_bytes(A.n, A.nnz, fs, vb, 4),
                          "moved_bytes_per_launch_ka": ka_bytes(A.n, A.nnz, fs, vb,
                                                                2 if m.info()["index16"] else 4)}),
              flush=True)
        return

    def solve(pol, R, maxit=5000, profile=False, vec16=0, variant=0):
        m.set_policy(pol)
        m.set_options(replace_period=R, fallback=False, profile=profile, vec16=vec16, variant=variant)
        xd.zero_()
        return m.solve(bd, xd, tol=tol, maxit=maxit)

    # warmup (also loads the code objects)
    for _ in range(args.warmup):
        solve(pol_mixed, 50)
        solve(pol_fp64, 0)
    torch.cuda.synchronize()

    # timed region: K mixed solves, each to a true relative residual <= tol
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = [solve(pol_mixed, 50) for _ in range(args.steps)]
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) * 1e3 / args.steps
    res = results[-1]
    for r in results:
        assert r["status"] == 0 and r["relres_true"] <= tol, r
    dev_ms = float(np.median([r["time_ms"] for r in results]))
    log(f"[bench] mixed: {res['iters']} it, relres {res['relres_true']:.3e}, device {dev_ms:.2f} ms, "
        f"wall {wall_ms:.2f} ms")

    # q52 (Table 1's quarter precision) matrix storage, same dot and update formats
    act_q52 = M.action(M.Q52, M.FP32, M.FP32)
    pol_q52 = M.Policy(kind=M.POLICY_FIXED, fixed_action=act_q52)
    solve(pol_q52, 50)
    q52_runs = [solve(pol_q52, 50) for _ in range(max(1, args.steps // 2))]
    rq = q52_runs[-1]
    assert rq["status"] == 0 and rq["relres_true"] <= tol, rq
    q52_ms = float(np.median([r["time_ms"] for r in q52_runs]))
    log(f"[bench] q52: {rq['iters']} it, relres {rq['relres_true']:.3e}, device {q52_ms:.2f} ms")

    # 16-bit vector storage: bf16 updates with r, p, x_lo in bf16 containers
    # against fp32 containers, 200 iterations of the same action
    act_b16 = M.action(M.BF16, M.FP32, M.BF16)
    pol_b16 = M.Policy(kind=M.POLICY_FIXED, fixed_action=act_b16)
    v16 = {}
    for v in (0, 1):
        solve(pol_b16, 50, maxit=200, vec16=v)
        rv = solve(pol_b16, 50, maxit=200, vec16=v, profile=True)
        pv = m.profile()
        it = pv["n_iter_slots"]
        v16[v] = {"iters": rv["iters"], "us_per_iteration": round(1e3 * rv["time_ms"] / rv["iters"], 2),
                  "ka_us": round(1e3 * pv["ka_iter_ms"] / it, 2), "kb_us": round(1e3 * pv["kb_iter_ms"] / it, 2),
                  "kx_us": round(1e3 * pv["kx_iter_ms"] / it, 2)}
        # plain timing (no events) of the same 200 iterations
        v16[v]["ms_200_iterations"] = round(float(np.median([solve(pol_b16, 50, maxit=200, vec16=v)["time_ms"]
                                                             for _ in range(3)])), 3)
    log(f"[bench] bf16 updates, fp32 vs bf16 containers: {v16}")

    fp64_runs = [solve(pol_fp64, 0) for _ in range(max(1, args.steps // 2))]
    r64 = fp64_runs[-1]
    assert r64["status"] == 0, r64
    fp64_ms = float(np.median([r["time_ms"] for r in fp64_runs]))
    log(f"[bench] fp64: {r64['iters']} it, relres {r64['relres_true']:.3e}, device {fp64_ms:.2f} ms")

    # single-reduction CG (two launches per iteration), the same actions
    sr = {}
    for name, pol, R in (("mixed", pol_mixed, 50), ("fp64", pol_fp64, 0)):
        solve(pol, R, variant=1)
        runs = [solve(pol, R, variant=1) for _ in range(max(1, args.steps // 2))]
        rs = runs[-1]
        assert rs["status"] == 0 and rs["relres_true"] <= tol, rs
        sr[name] = {"ms": round(float(np.median([r["time_ms"] for r in runs])), 3), "iters": rs["iters"],
                    "n_replace": rs["n_replace"], "relres_true": rs["relres_true"]}
    sr["mixed"]["speedup_vs_three_launch_mixed"] = round(dev_ms / sr["mixed"]["ms"], 3)
    sr["mixed"]["speedup_vs_fp64"] = round(fp64_ms / sr["mixed"]["ms"], 3)
    sr["fp64"]["speedup_vs_three_launch_fp64"] = round(fp64_ms / sr["fp64"]["ms"], 3)
    log(f"[bench] single-reduction CG: {sr}")

    # pipelined CG (w = A r and z = A s by recurrence as well); its recurrences
    # need replacements every 20 iterations with the mixed action
    pc = {}
    for name, pol, R in (("mixed", pol_mixed, 20), ("fp64", pol_fp64, 50)):
        solve(pol, R, variant=2)
        runs = [solve(pol, R, variant=2) for _ in range(max(1, args.steps // 2))]
        rs = runs[-1]
        pc[name] = {"replace_period": R, "ms": round(float(np.median([r["time_ms"] for r in runs])), 3),
                    "iters": rs["iters"], "status": rs["status"], "n_replace": rs["n_replace"],
                    "relres_true": rs["relres_true"]}
    pc["mixed"]["speedup_vs_three_launch_mixed"] = round(dev_ms / pc["mixed"]["ms"], 3)
    pc["fp64"]["speedup_vs_three_launch_fp64"] = round(fp64_ms / pc["fp64"]["ms"], 3)
    log(f"[bench] pipelined CG: {pc}")

    # profiled solves: HIP events around every launch of the same kernels
    rp = solve(pol_mixed, 50, profile=True)
    prof = m.profile()
    rp64 = solve(pol_fp64, 0, profile=True)
    prof64 = m.profile()
    solve(pol_q52, 50, profile=True)
    profq = m.profile()
    k1_q_us = profq["ka_iter_ms"] / profq["n_iter_slots"] * 1e3
    k1_us = prof["ka_iter_ms"] / prof["n_iter_slots"] * 1e3
    k2_us = prof["kb_iter_ms"] / prof["n_iter_slots"] * 1e3
    k3_us = prof["kx_iter_ms"] / prof["n_iter_slots"] * 1e3
    k1_64_us = prof64["ka_iter_ms"] / prof64["n_iter_slots"] * 1e3
    k2_64_us = prof64["kb_iter_ms"] / prof64["n_iter_slots"] * 1e3
    k3_64_us = prof64["kx_iter_ms"] / prof64["n_iter_slots"] * 1e3
    idx_bytes = 2 if m.info()["index16"] else 4
    bytes_k1 = ka_bytes(A.n, A.nnz, M.BF16, 4, 4)            # algorithmic: int32 column indices
    bytes_k1_moved = ka_bytes(A.n, A.nnz, M.BF16, 4, idx_bytes)   # what the kernel streams
    bytes_k1_64 = ka_bytes(A.n, A.nnz, M.FP64, 8, 4)
    bytes_k2 = 6 * A.n * 4      # p, q, r, x_lo read; r, x_lo written
    bytes_k2_64 = 6 * A.n * 8
    bytes_k3 = 3 * A.n * 4      # p, r read; p written
    bytes_k3_64 = 3 * A.n * 8
    achieved = bytes_k1 / (k1_us * 1e-6) / 1e9
    log(f"[bench] profile mixed: KA {k1_us:.2f} us ({achieved:.0f} GB/s)  KB {k2_us:.2f} us  KX {k3_us:.2f} us  "
        f"profiled solve {rp['time_ms']:.2f} ms; fp64 KA {k1_64_us:.2f} us KB {k2_64_us:.2f} us "
        f"KX {k3_64_us:.2f} us")

    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        tr = json.load(open(TRAFFIC_FILE))
        if tr.get("kernel_hash") == kernel_hash() and tr.get("workload") == A.name:
            traffic = tr.get("bytes_per_launch")

    out = {
        "metric": METRIC,
        "value": round(dev_ms, 3),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall_ms, 3),
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "bf16/f32/f64",
        "data": "synthetic",
        "config": {
            "workload": f"3D 7-point Laplacian {args.N}^3 (n={A.n}, nnz={A.nnz}), b~U[-1,1] seed 2, x0=0, "
                        f"tol 1e-8 true fp64 relres; mixed action (SpMV bf16/fp32-acc, dot fp32, axpy fp32), "
                        f"fp64 replacement every 50 iterations",
            "solver": "mixed-precision CG, fixed policy", "device": dev_name,
        },
        "iters": res["iters"],
        "relres_true": res["relres_true"],
        "fp64_ms": round(fp64_ms, 3),
        "fp64_iters": r64["iters"],
        "speedup_vs_fp64": round(fp64_ms / dev_ms, 3),
        "setup_ms": round(setup_ms, 1),
        "roofline": {
            "bound": "hbm",
            "kernel": "k_a: CSR SpMV (bf16 values, " + ("16-bit column deltas" if idx_bytes == 2 else "int32 columns")
                      + ", fp32 accumulation) with the fused p.q partial",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "bytes_per_launch": bytes_k1,
            "avg_launch_us": round(k1_us, 3),
            "launches": prof["n_iter_slots"],
            "moved_bytes_per_launch": bytes_k1_moved,
            "achieved_on_moved_bytes": round(bytes_k1_moved / (k1_us * 1e-6) / 1e9, 1),
            "frac_on_moved_bytes": round(bytes_k1_moved / (k1_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
        },
        "kernels": {
            "kb_axpy_dot": {"avg_us": round(k2_us, 3), "GB/s": round(bytes_k2 / (k2_us * 1e-6) / 1e9, 1)},
            "kx_direction": {"avg_us": round(k3_us, 3), "GB/s": round(bytes_k3 / (k3_us * 1e-6) / 1e9, 1)},
            "ka_fp64": {"avg_us": round(k1_64_us, 3), "GB/s": round(bytes_k1_64 / (k1_64_us * 1e-6) / 1e9, 1)},
            "kb_fp64": {"avg_us": round(k2_64_us, 3), "GB/s": round(bytes_k2_64 / (k2_64_us * 1e-6) / 1e9, 1)},
            "kx_fp64": {"avg_us": round(k3_64_us, 3), "GB/s": round(bytes_k3_64 / (k3_64_us * 1e-6) / 1e9, 1)},
            "profiled_solve_ms": round(rp["time_ms"], 3),
        },
        "single_reduction": dict(
            variant="Chronopoulos-Gear CG: SpMV w = A r with both inner products fused, s = A p by "
                    "recurrence, two launches per iteration", **sr),
        "pipelined": dict(
            variant="Ghysels-Vanroose CG: SpMV q = A w independent of the inner products, w = A r and "
                    "z = A s by recurrence, six vector updates, two launches per iteration", **pc),
        "vector_storage_16bit": {
            "action": "SpMV bf16, dot fp32, updates bf16, R=50, 200 iterations",
            "fp32_containers": v16[0], "bf16_containers": v16[1],
            "speedup": round(v16[0]["ms_200_iterations"] / v16[1]["ms_200_iterations"], 3)},
        "q52_storage": {
            "action": "SpMV in q52 storage (row-scaled, fp32 accumulation), dot fp32, axpy fp32, R=50",
            "ms": round(q52_ms, 3), "iters": rq["iters"], "relres_true": rq["relres_true"],
            "speedup_vs_fp64": round(fp64_ms / q52_ms, 3),
            "ka_avg_us": round(k1_q_us, 3),
            "ka_GB/s_algorithmic": round(ka_bytes(A.n, A.nnz, 4, 4, 4) / (k1_q_us * 1e-6) / 1e9, 1),
            "ka_GB/s_moved": round(ka_bytes(A.n, A.nnz, 4, 4, idx_bytes) / (k1_q_us * 1e-6) / 1e9, 1),
        },
    }

    if not args.no_learned:
        # Q-table trained on the device (Algorithm 1) over small seeded systems of the
        # training family, then used greedily on this workload.
        t0 = time.time()
        P_l, tr = train_qtable(M, build_systems(M, W, torch, range(100, 112), n_hi=1e5), episodes=3,
                               maxit=1000, cost="C1")
        t_train = time.time() - t0
        greedy = M.Policy(kind=M.POLICY_QTABLE, cost="C1")   # the trained table, no exploration
        greedy.set_qtable(P_l.qtable())
        m.set_policy(greedy)
        m.set_options(replace_period=50, fallback=True)
        lr_runs = []
        for _ in range(max(1, args.steps // 2) + 1):
            xd.zero_()
            lr_runs.append(m.solve(bd, xd, tol=tol, maxit=5000))
        rl = lr_runs[-1]
        h = m.history()
        out["learned"] = {"policy": "Q-table, C1 costs, trained on 12 seeded systems x 3 episodes "
                                    "(2D/3D Laplacians, random SPD, n <= 1e5)",
                          "ms": round(float(np.median([r["time_ms"] for r in lr_runs[1:]])), 3),
                          "iters": rl["iters"], "status": rl["status"], "relres_true": rl["relres_true"],
                          "train_s": round(t_train, 1), "train_episodes": len(tr),
                          "action_mix": mix_of(M, h["actions"]),
                          "speedup_vs_fp64": round(fp64_ms / float(np.median([r["time_ms"] for r in lr_runs[1:]])), 3)}
        log(f"[bench] learned: {out['learned']}")
        # the same table restricted to the SpMV format (dots and updates in
        # fp32; the other actions masked), a labelled variation
        keep = [M.action(fs, M.FP32, M.FP32) for fs in (M.FP16, M.BF16, M.FP32, M.FP64)]
        qm = P_l.qtable().copy()
        qm[:, [a for a in range(64) if a not in keep]] = -1e300
        gm = M.Policy(kind=M.POLICY_QTABLE, cost="C1")
        gm.set_qtable(qm)
        m.set_policy(gm)
        m.set_options(replace_period=50, fallback=True)
        sp_runs = []
        for _ in range(max(1, args.steps // 2) + 1):
            xd.zero_()
            sp_runs.append(m.solve(bd, xd, tol=tol, maxit=5000))
        rs = sp_runs[-1]
        ms_sp = float(np.median([r["time_ms"] for r in sp_runs[1:]]))
        out["learned"]["spmv_only"] = {"policy": "the same table, SpMV format learned, dots and updates in fp32",
                                       "ms": round(ms_sp, 3), "iters": rs["iters"], "status": rs["status"],
                                       "relres_true": rs["relres_true"], "action_mix": mix_of(M, m.history()["actions"]),
                                       "speedup_vs_fp64": round(fp64_ms / ms_sp, 3)}
        log(f"[bench] learned, SpMV only: {out['learned']['spmv_only']}")
        m.set_policy(pol_mixed)

    if not args.no_rspd:
        t0 = time.time()
        R = W.random_spd(1_000_000, 3, W.spread_for_kappa(1e6))
        bR = W.rhs(R.n, 4)
        log(f"[bench] generated random SPD n={R.n} nnz={R.nnz} in {time.time() - t0:.1f}s")
        mR = M.Matrix(R)
        bRd = torch.from_numpy(bR).cuda()
        xRd = torch.zeros(R.n, dtype=torch.float64, device="cuda")
        rr = {}
        for name, pol, Rp in (("mixed", pol_mixed, 50), ("fp64", pol_fp64, 0)):
            mR.set_policy(pol)
            mR.set_options(replace_period=Rp, fallback=False)
            xRd.zero_()
            r = mR.solve(bRd, xRd, tol=tol, maxit=60000)
            rr[name] = {"ms": round(r["time_ms"], 3), "iters": r["iters"], "status": r["status"],
                        "relres_true": r["relres_true"]}
            log(f"[bench] rspd {name}: {r}")
        out["random_spd"] = {"n": R.n, "nnz": R.nnz, **rr,
                             "speedup_vs_fp64": round(rr["fp64"]["ms"] / rr["mixed"]["ms"], 3)}
        # the SpMV's time per launch against the random-access floor of its columns
        mR.set_policy(pol_mixed)
        mR.set_options(replace_period=50, fallback=False, profile=True)
        xRd.zero_()
        mR.solve(bRd, xRd, tol=tol, maxit=200)
        prR = mR.profile()
        ka_r_us = prR["ka_iter_ms"] / prR["n_iter_slots"] * 1e3
        p32 = torch.from_numpy(np.random.default_rng(9).standard_normal(R.n).astype(np.float32)).cuda()
        floor_us = mR.gather_floor(p32, 20)
        out["random_spd"]["ka_us"] = round(ka_r_us, 2)
        out["random_spd"]["ka_GB/s_algorithmic"] = round(ka_bytes(R.n, R.nnz, M.BF16, 4, 4) / (ka_r_us * 1e-6) / 1e9, 1)
        out["random_spd"]["gather_floor_us"] = round(floor_us, 2)
        out["random_spd"]["ka_vs_gather_floor"] = round(floor_us / ka_r_us, 3)
        log(f"[bench] rspd KA {ka_r_us:.2f} us, flat gather floor {floor_us:.2f} us")
        # the same system with the Jacobi preconditioner (section 3's z = M^-1 r)
        pj = {}
        for name, pol, Rp in (("mixed", pol_mixed, 50), ("fp64", pol_fp64, 0)):
            mR.set_policy(pol)
            mR.set_options(replace_period=Rp, fallback=False, precond=1)
            runs = []
            for _ in range(3):
                xRd.zero_()
                runs.append(mR.solve(bRd, xRd, tol=tol, maxit=60000))
            r = runs[-1]
            assert r["status"] == 0 and r["relres_true"] <= tol, r
            pj[name] = {"ms": round(float(np.median([q["time_ms"] for q in runs])), 3), "iters": r["iters"],
                        "status": r["status"], "relres_true": r["relres_true"]}
            log(f"[bench] rspd jacobi {name}: {r}")
        out["random_spd"]["jacobi"] = {**pj, "speedup_vs_fp64_jacobi": round(pj["fp64"]["ms"] / pj["mixed"]["ms"], 3),
                                       "speedup_vs_unpreconditioned_fp64": round(rr["fp64"]["ms"] / pj["mixed"]["ms"], 1)}

    # the small fp64 case: plain fp64 CG on the 2D 5-point Laplacian 64x64
    # (n = 4096), b ~ U[-1,1] seed 1, x0 = 0, tol 1e-8, maxit 2000; at this
    # size an iteration is launch-bound, which the two-launch variant shows
    S = W.laplacian_2d(64)
    msm = M.Matrix(S)
    bsm = torch.from_numpy(W.rhs(S.n, 1)).cuda()
    small = {"n": S.n, "nnz": S.nnz}
    for name, variant in (("three_launch", 0), ("single_reduction", 1)):
        msm.set_policy(pol_fp64)
        msm.set_options(replace_period=0, fallback=False, variant=variant)
        runs = []
        for _ in range(4):
            xsm = torch.zeros(S.n, dtype=torch.float64, device="cuda")
            runs.append(msm.solve(bsm, xsm, tol=1e-8, maxit=2000))
        r = runs[-1]
        ms_small = float(np.median([q["time_ms"] for q in runs[1:]]))
        small[name] = {"ms": round(ms_small, 3), "iters": r["iters"], "status": r["status"],
                       "relres_true": r["relres_true"], "us_per_iteration": round(1e3 * ms_small / max(1, r["iters"]), 2)}
    log(f"[bench] 2D Laplacian 64^2 fp64: {small}")
    out["laplacian_2d_64_fp64"] = small

    if not args.no_cpu:
        import oracle as O

        host = {"cpu_model": cpu_model(), "cores_available": len(os.sched_getaffinity(0)),
                "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}
        # the oracle's plain fp64 CG (native double, no emulation), single-threaded,
        # on the whole workload, run to the same tolerance
        t0 = time.perf_counter()
        _, it_p, rr_p = O.cg_plain(A, b, tol=tol, maxit=5000)
        t_p = time.perf_counter() - t0
        log(f"[bench] oracle plain fp64 CG: {it_p} it in {t_p:.2f} s (1 thread)")
        # the same method on every host core (fixed-chunk, in-order reductions)
        t0 = time.perf_counter()
        _, it_o, rr_o, th = O.cg_openmp(A, b, tol=tol, maxit=5000)
        t_o = time.perf_counter() - t0
        log(f"[bench] OpenMP fp64 CG: {it_o} it in {t_o:.2f} s ({th} threads)")
        # the emulated mixed oracle: its shadow setup (a solve with maxit 0) is
        # subtracted; this is a parity tool, not a speed baseline
        sample_it = 20
        t0 = time.perf_counter()
        O.cg(A, b, tol=1e-30, maxit=0, policy=O.OraclePolicy(fixed_action=act_mixed), replace_period=50)
        t_setup = time.perf_counter() - t0
        t0 = time.perf_counter()
        O.cg(A, b, tol=1e-30, maxit=sample_it, policy=O.OraclePolicy(fixed_action=act_mixed), replace_period=50)
        t_em = time.perf_counter() - t0 - t_setup
        out["cpu_baseline"] = {
            "value": round(t_p * 1e3, 1),
            "unit": "ms",
            "cores": 1,
            "kind": "oracle",
            "sample": f"the whole workload: the oracle's plain fp64 CG (native double, no emulation) on the "
                      f"3D Laplacian {args.N}^3 from x0 = 0, run to convergence ({it_p} iterations, recursive "
                      f"relres {rr_p:.2e}), single-threaded; the GPU's fp64 CG takes {r64['iters']} iterations",
            "vs_gpu_fp64": round(t_p * 1e3 / fp64_ms, 1),
            "vs_gpu_mixed": round(t_p * 1e3 / dev_ms, 1),
            "openmp": {"value": round(t_o * 1e3, 1), "unit": "ms", "cores": th, "iters": it_o,
                       "relres": rr_o, "kind": "fp64 CG, OpenMP row-parallel SpMV and updates, "
                                                "fixed 8192-row chunk sums added in chunk order"},
            "emulated_mixed": {"label": "emulation: not a speed baseline",
                               "ms_per_iteration": round(t_em / sample_it * 1e3, 2),
                               "sample": f"{sample_it} iterations of the oracle's emulated mixed CG (same "
                                         f"action), shadow setup ({t_setup:.2f} s) excluded"},
            "host": host,
        }
        log(f"[bench] oracle emulated mixed: {t_em / sample_it * 1e3:.1f} ms/it (setup {t_setup:.2f} s excluded)")

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
