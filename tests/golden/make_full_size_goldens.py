"""Writes tests/golden/full_size_<name>.json: the oracle's whole mixed-precision
solve (section 3's recurrences with the per-iteration precisions of section 4.2)
on the benchmark's two full-size systems, for the exact comparison in
tests/test_gpu_full_size.py.  Calls only oracle/ and workloads/ (seeded inputs).

    python tests/golden/make_full_size_goldens.py lap3d_128     # ~2 min on one core
    python tests/golden/make_full_size_goldens.py rspd_1e6      # ~45 min on one core
"""
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402

ACTION = 16 * 1 + 4 * 2 + 2          # SpMV bf16 storage, dot fp32, axpy fp32


def system(name):
    if name == "lap3d_128":
        A = W.laplacian_3d(128)
        return A, W.rhs(A.n, 2), 5000
    if name == "rspd_1e6":
        A = W.random_spd(1_000_000, 3, W.spread_for_kappa(1e6))
        return A, W.rhs(A.n, 4), 60000
    raise SystemExit(f"unknown system {name}")


def sha(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def main(name):
    t0 = time.time()
    A, b, maxit = system(name)
    print(f"{name}: n={A.n} nnz={A.nnz} generated in {time.time() - t0:.0f}s", flush=True)
    t0 = time.time()
    x, info = O.cg(A, b, tol=1e-8, maxit=maxit, policy=O.OraclePolicy(fixed_action=ACTION),
                   replace_period=50, fallback=False)
    secs = time.time() - t0
    out = {
        "system": name, "n": A.n, "nnz": A.nnz, "action": ACTION, "tol": 1e-8, "maxit": maxit,
        "replace_period": 50, "fallback": False,
        "status": info["status"], "iters": info["iters"], "n_replace": info["n_replace"],
        "fallback_at": info["fallback_at"], "relres_true": info["relres_true"].hex(),
        "rep_k": info["rep_k"].tolist(), "rep_rho": [float(v).hex() for v in info["rep_rho"]],
        "sha256_rho": sha(info["rho"].astype(np.float64)), "sha256_actions": sha(info["actions"].astype(np.uint8)),
        "sha256_x": sha(x.astype(np.float64)), "oracle_seconds": round(secs, 1),
    }
    path = os.path.join(HERE, f"full_size_{name}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(f"{name}: status {info['status']} iters {info['iters']} relres {info['relres_true']:.3e} "
          f"in {secs:.0f}s -> {path}", flush=True)


if __name__ == "__main__":
    for nm in sys.argv[1:] or ["lap3d_128", "rspd_1e6"]:
        main(nm)
