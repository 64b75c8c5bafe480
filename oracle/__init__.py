"""ctypes shim over the C oracle (mpcg_oracle.c).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg load this module; the product path never does.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from decimal import Decimal, getcontext

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mpcg_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

F16, BF16, F32, F64, Q52, TF32 = 0, 1, 2, 3, 4, 5
ORDER_PAIRWISE, ORDER_SEQ = 0, 1
POL_FIXED, POL_QTABLE, POL_QTRAIN, POL_MLP = 0, 1, 2, 3
FL_REPLACED, FL_EXPLORED, FL_FALLBACK, FL_SWITCH = 1, 2, 4, 8


OMP_SRC = os.path.join(HERE, "cg_openmp.c")
OMP_LIB = os.path.join(HERE, "libcgomp.so")


def build() -> str:
    """Compile the oracle with gcc (ISO C, no contraction, no fast math), and the
    multi-core fp64 CG speed baseline beside it (OpenMP)."""
    cmd = ["gcc", "-std=c11", "-O2", "-Wall", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-o", LIB + ".tmp", SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    cmd = ["gcc", "-std=c11", "-O2", "-Wall", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-o", OMP_LIB + ".tmp", OMP_SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(OMP_LIB + ".tmp", OMP_LIB)
    return LIB


_omp = None


def cg_openmp(A, b, tol=1e-8, maxit=1000):
    """Plain fp64 CG on every host core (speed baseline).  Returns (x, iters, relres, threads)."""
    global _omp
    if _omp is None:
        if not os.path.exists(OMP_LIB) or os.path.getmtime(OMP_LIB) < os.path.getmtime(OMP_SRC):
            build()
        L = C.CDLL(OMP_LIB)
        dp, ip = C.POINTER(C.c_double), C.POINTER(C.c_int32)
        L.cgomp_solve.restype = C.c_int
        L.cgomp_solve.argtypes = [C.c_int64, ip, ip, dp, dp, dp, C.c_double, C.c_int32, ip, dp]
        _omp = L
    x = np.zeros(A.n)
    it = C.c_int32(0)
    rr = C.c_double(0.0)
    th = _omp.cgomp_solve(A.n, _p(_i32(A.row_ptr), C.c_int32), _p(_i32(A.col), C.c_int32), _p(_f64(A.val)),
                          _p(_f64(b)), _p(x), tol, maxit, C.byref(it), C.byref(rr))
    return x, it.value, rr.value, th


class Policy(C.Structure):
    _fields_ = [
        ("kind", C.c_int32), ("fixed_action", C.c_int32),
        ("t_bin", C.c_int32), ("b_it", C.c_int32), ("b_res", C.c_int32), ("w_stag", C.c_int32),
        ("res_edges", C.c_double * 16),
        ("q", C.POINTER(C.c_double)),
        ("lr", C.c_double), ("gamma", C.c_double),
        ("w1", C.c_double), ("w2", C.c_double), ("w3", C.c_double), ("eps_min", C.c_double),
        ("cost", C.c_double * 4),
        ("epsilon", C.c_double),
        ("seed", C.c_uint64), ("episode", C.c_int64),
        ("w1m", C.POINTER(C.c_float)), ("b1m", C.POINTER(C.c_float)),
        ("w2m", C.POINTER(C.c_float)), ("b2m", C.POINTER(C.c_float)),
        ("w3m", C.POINTER(C.c_float)), ("b3m", C.POINTER(C.c_float)),
        ("replace_period", C.c_int32), ("decision_period", C.c_int32),
        ("per_op", C.c_int32), ("nfmt", C.c_int32), ("cost_tf32", C.c_double),
    ]


class Params(C.Structure):
    _fields_ = [("tol", C.c_double), ("maxit", C.c_int32), ("replace_period", C.c_int32),
                ("fallback", C.c_int32), ("dot_order", C.c_int32), ("precond", C.c_int32),
                ("stop_rule", C.c_int32), ("rho_fp64", C.c_int32), ("emulate", C.c_int32),
                ("vec16", C.c_int32)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("n_replace", C.c_int32),
                ("fallback_at", C.c_int32), ("relres_true", C.c_double), ("cost_sum", C.c_double)]


class Hist(C.Structure):
    _fields_ = [
        ("hist_rho", C.POINTER(C.c_double)), ("hist_act", C.POINTER(C.c_uint8)),
        ("hist_flag", C.POINTER(C.c_uint8)), ("rep_k", C.POINTER(C.c_int32)),
        ("rep_rho", C.POINTER(C.c_double)), ("rep_cap", C.c_int32), ("roll_cap", C.c_int32),
        ("roll_feat", C.POINTER(C.c_float)), ("roll_next", C.POINTER(C.c_float)),
        ("roll_act", C.POINTER(C.c_int32)), ("roll_rew", C.POINTER(C.c_float)),
        ("roll_done", C.POINTER(C.c_uint8)), ("roll_n", C.c_int32), ("dump_cap", C.c_int32),
        ("hist_alpha", C.POINTER(C.c_double)), ("hist_beta", C.POINTER(C.c_double)),
        ("dump_p", C.POINTER(C.c_double)), ("dump_r", C.POINTER(C.c_double)),
        ("dump_s", C.POINTER(C.c_double)), ("dump_w", C.POINTER(C.c_double)),
        ("dump_z", C.POINTER(C.c_double)),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = C.CDLL(LIB)
        dp, ip, i64, d = C.POINTER(C.c_double), C.POINTER(C.c_int32), C.c_int64, C.c_double
        L.orc_rd.restype = d
        L.orc_rd.argtypes = [d, C.c_int]
        L.orc_rd_array.argtypes = [dp, dp, i64, C.c_int]
        L.orc_row_exp.restype = C.c_int
        L.orc_row_exp.argtypes = [dp, i64]
        L.orc_shadows.argtypes = [i64, ip, ip, dp, dp, dp, dp, ip]
        L.orc_spmv.argtypes = [i64, ip, ip, dp, C.c_int, C.c_int, dp, dp]
        L.orc_shadow_q52.argtypes = [i64, ip, ip, dp, dp, ip]
        L.orc_shadow_tf32.argtypes = [i64, ip, ip, dp, dp]
        L.orc_act_decode.argtypes = [C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.orc_jacobi_inverse.argtypes = [i64, ip, ip, dp, C.POINTER(C.c_float)]
        L.orc_residual.argtypes = [i64, ip, ip, dp, dp, dp, dp]
        L.orc_dot.restype = d
        L.orc_dot.argtypes = [i64, dp, dp, C.c_int, C.c_int]
        L.orc_axpy.argtypes = [i64, d, dp, dp, C.c_int]
        L.orc_xpay.argtypes = [i64, d, dp, dp, C.c_int]
        L.orc_log10.restype = d
        L.orc_log10.argtypes = [d]
        L.orc_uniform.restype = d
        L.orc_uniform.argtypes = [C.c_uint64] * 4
        L.orc_mix64.restype = C.c_uint64
        L.orc_mix64.argtypes = [C.c_uint64]
        L.orc_stag.restype = C.c_int
        L.orc_stag.argtypes = [dp, i64, C.c_int]
        L.orc_stagnated.restype = C.c_int
        L.orc_stagnated.argtypes = [C.c_int, dp]
        L.orc_state.restype = C.c_int
        L.orc_state.argtypes = [C.POINTER(Policy), i64, d, C.c_int]
        L.orc_reward.restype = d
        L.orc_reward.argtypes = [C.POINTER(Policy), C.c_int, d, C.c_int]
        L.orc_gelu.restype = C.c_float
        L.orc_gelu.argtypes = [C.c_float]
        L.orc_mlp_logits.argtypes = [C.POINTER(Policy), C.POINTER(C.c_float), C.POINTER(C.c_float)]
        L.orc_mlp_features.argtypes = [C.POINTER(Policy), i64, dp, C.c_int, d, C.c_int,
                                       C.POINTER(C.c_float)]
        L.orc_cg.restype = C.c_int
        L.orc_cg.argtypes = [i64, ip, ip, dp, dp, dp, dp, C.POINTER(Params), C.POINTER(Policy),
                             C.POINTER(Result), C.POINTER(Hist)]
        L.orc_cg_plain.restype = C.c_int
        L.orc_cg_sr.argtypes = [i64, ip, ip, dp, dp, dp, dp, C.c_int, C.POINTER(Params), C.POINTER(Result),
                                C.POINTER(Hist)]
        L.orc_cg_pipe.argtypes = L.orc_cg_sr.argtypes
        L.orc_cg_plain.argtypes = [i64, ip, ip, dp, dp, dp, d, C.c_int32, ip, dp]
        _lib = L
    return _lib


def _p(a, t=C.c_double):
    return a.ctypes.data_as(C.POINTER(t))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


# ---------------------------------------------------------------- elementary ops
def rd(x, fmt: int):
    x = _f64(np.atleast_1d(x))
    y = np.empty_like(x)
    lib().orc_rd_array(_p(x), _p(y), x.size, fmt)
    return y


def row_exp(vals) -> int:
    v = _f64(vals)
    return lib().orc_row_exp(_p(v), v.size)


def shadows(A):
    nnz = A.nnz
    s32, sb, sh = np.empty(nnz), np.empty(nnz), np.empty(nnz)
    e = np.empty(A.n, dtype=np.int32)
    lib().orc_shadows(A.n, _p(_i32(A.row_ptr), C.c_int32), _p(_i32(A.col), C.c_int32),
                      _p(_f64(A.val)), _p(s32), _p(sb), _p(sh), _p(e, C.c_int32))
    return s32, sb, sh, e


def shadow_q52(A):
    """(q52 shadow values as float64, row exponents) of the CSR matrix A."""
    v = np.empty(A.nnz)
    e = np.empty(A.n, dtype=np.int32)
    lib().orc_shadow_q52(A.n, _p(_i32(A.row_ptr), C.c_int32), _p(_i32(A.col), C.c_int32), _p(_f64(A.val)),
                         _p(v), _p(e, C.c_int32))
    return v, e


def shadow_tf32(A):
    """tf32 shadow values (as float64) of the CSR matrix A."""
    v = np.empty(A.nnz)
    lib().orc_shadow_tf32(A.n, _p(_i32(A.row_ptr), C.c_int32), _p(_i32(A.col), C.c_int32), _p(_f64(A.val)), _p(v))
    return v


def spmv(A, p, fs: int, tier64: int):
    p = _f64(p)
    q = np.empty(A.n)
    lib().orc_spmv(A.n, _p(_i32(A.row_ptr), C.c_int32), _p(_i32(A.col), C.c_int32),
                   _p(_f64(A.val)), fs, tier64, _p(p), _p(q))
    return q


def residual(A, b, x):
    r = np.empty(A.n)
    lib().orc_residual(A.n, _p(_i32(A.row_ptr), C.c_int32), _p(_i32(A.col), C.c_int32),
                       _p(_f64(A.val)), _p(_f64(b)), _p(_f64(x)), _p(r))
    return r


def dot(u, v, fd: int, order: int = ORDER_PAIRWISE) -> float:
    u, v = _f64(u), _f64(v)
    return lib().orc_dot(u.size, _p(u), _p(v), fd, order)


def axpy(alpha: float, u, y, fa: int):
    y = _f64(y).copy()
    lib().orc_axpy(y.size, alpha, _p(_f64(u)), _p(y), fa)
    return y


def xpay(beta: float, r, p, fa: int):
    p = _f64(p).copy()
    lib().orc_xpay(p.size, beta, _p(_f64(r)), _p(p), fa)
    return p


def log10(x: float) -> float:
    return lib().orc_log10(x)


def stag_flag(hist_rho, k: int, W: int) -> int:
    """The state's stagnation flag stag_k on the history rho_0..rho_k."""
    h = _f64(hist_rho)
    return lib().orc_stag(_p(h), k, W)


def stagnated(m: int, last3) -> int:
    """The fallback trigger at the m-th replacement: last3 = true rho at m-2, m-1, m."""
    t = _f64(last3)
    return lib().orc_stagnated(m, _p(t))


def uniform(seed: int, episode: int, k: int, stream: int) -> float:
    return lib().orc_uniform(seed, episode, k, stream)


def mix64(z: int) -> int:
    return lib().orc_mix64(z)


def gelu(x: float) -> float:
    return lib().orc_gelu(x)


# ---------------------------------------------------------------- policy setup
def residual_edges(b_res: int = 10, eps_min_exp: int = 16):
    """Nearest doubles to 10^(-j*delta), j = 1..b_res-1, delta = eps_min_exp / b_res."""
    getcontext().prec = 60
    out = []
    for j in range(1, b_res):
        e = Decimal(-eps_min_exp * j) / Decimal(b_res)
        out.append(float(Decimal(10) ** e))
    return out


# c(fp16), c(bf16), c(fp32), c(fp64), c(tf32) (section 5)
COSTS = {"C1": (0.8, 0.6, 1.0, 2.0, 0.8), "C2": (0.5, 0.4, 1.5, 3.0, 0.5)}


def action(fs, fd, fa):
    """Action code of (f_s, f_d, f_a): 16 f_s + 4 f_d + f_a over the four
    arithmetic formats; with tf32 in a slot, 128 + 25 d_s + 5 d_d + d_a over the
    digits (fp16, bf16, fp32, fp64, tf32) = 0..4."""
    d = [4 if f == TF32 else f for f in (fs, fd, fa)]
    if 4 in d:
        return 128 + 25 * d[0] + 5 * d[1] + d[2]
    return 16 * d[0] + 4 * d[1] + d[2]


def act_decode(a):
    """(f_s, f_d, f_a) of an action code, as the oracle's solver reads it."""
    fs, fd, fa = C.c_int(), C.c_int(), C.c_int()
    lib().orc_act_decode(int(a), C.byref(fs), C.byref(fd), C.byref(fa))
    return fs.value, fd.value, fa.value


class OraclePolicy:
    """Owns the arrays behind a Policy struct."""

    def __init__(self, kind=POL_FIXED, fixed_action=63, q=None, t_bin=1000, b_it=5,
                 b_res=10, w_stag=10, lr=0.1, gamma=0.9, w=(1.0, 0.1, 10.0), eps_min=1e-16,
                 cost="C1", epsilon=0.0, seed=0, episode=0, mlp=None, replace_period=50, decision_period=1,
                 per_op=0, nfmt=4):
        self.s = Policy()
        s = self.s
        s.kind, s.fixed_action = kind, fixed_action
        s.t_bin, s.b_it, s.b_res, s.w_stag = t_bin, b_it, b_res, w_stag
        # section 4.1: delta = -log10(eps_min) / r with eps_min a power of ten
        for i, e in enumerate(residual_edges(b_res, int(round(-math.log10(eps_min))))):
            s.res_edges[i] = e
        n_states = b_res * b_it * 2
        self.q = _f64(np.zeros((n_states, 64)) if q is None else q).copy()
        s.q = _p(self.q)
        s.lr, s.gamma = lr, gamma
        s.w1, s.w2, s.w3 = w
        s.eps_min = eps_min
        costs = COSTS[cost] if isinstance(cost, str) else cost
        for i in range(4):
            s.cost[i] = costs[i]
        s.cost_tf32 = costs[4] if len(costs) > 4 else costs[0]
        s.nfmt = int(nfmt)
        s.epsilon, s.seed, s.episode = epsilon, seed, episode
        s.replace_period = replace_period
        s.decision_period = decision_period
        s.per_op = int(per_op)
        self.mlp = None
        if mlp is not None:
            self.set_mlp(mlp)

    def set_mlp(self, mlp):
        """mlp: dict of float32 arrays W1[128,16], b1, W2[128,128], b2, W3[64,128], b3."""
        self.mlp = {k: np.ascontiguousarray(v, dtype=np.float32) for k, v in mlp.items()}
        s, m = self.s, self.mlp
        s.w1m, s.b1m = _p(m["W1"], C.c_float), _p(m["b1"], C.c_float)
        s.w2m, s.b2m = _p(m["W2"], C.c_float), _p(m["b2"], C.c_float)
        s.w3m, s.b3m = _p(m["W3"], C.c_float), _p(m["b3"], C.c_float)

    def reward(self, action, rho, terminal):
        return lib().orc_reward(C.byref(self.s), action, rho, int(terminal))

    def state(self, k, rho, stag):
        return lib().orc_state(C.byref(self.s), k, rho, int(stag))

    def mlp_logits(self, feat):
        f = np.ascontiguousarray(feat, dtype=np.float32)
        out = np.empty(64, dtype=np.float32)
        lib().orc_mlp_logits(C.byref(self.s), _p(f, C.c_float), _p(out, C.c_float))
        return out

    def mlp_features(self, k, hist_rho, stag, last_true, prev_action):
        h = _f64(hist_rho)
        out = np.empty(16, dtype=np.float32)
        lib().orc_mlp_features(C.byref(self.s), k, _p(h), int(stag), last_true, prev_action,
                               _p(out, C.c_float))
        return out


def jacobi_inverse(A):
    """The Jacobi preconditioner's inverse diagonal as stored (float32)."""
    out = np.empty(A.n, dtype=np.float32)
    lib().orc_jacobi_inverse(A.n, _p(_i32(A.row_ptr), C.c_int32), _p(_i32(A.col), C.c_int32), _p(_f64(A.val)),
                             _p(out, C.c_float))
    return out


def cg(A, b, x0=None, tol=1e-8, maxit=1000, policy: OraclePolicy | None = None,
       replace_period=0, fallback=False, order=ORDER_PAIRWISE, roll_cap=0, dump=0, precond=0, stop_rule=0,
       rho_fp64=0, emulate=0, vec16=0):
    """Run the oracle solver (precond 1: Jacobi; stop_rule 1: the paper's
    termination, recursive rho < tol with k >= 10; rho_fp64 1: rho from an
    fp64 r.r; emulate 1: the paper's reading, fp64 operations whose results are
    rounded to the operation's format; vec16 1: bf16 containers for r, p and
    x_lo when the updates are bf16).  Returns (x, info dict with histories)."""
    n = A.n
    b = _f64(b)
    x0 = np.zeros(n) if x0 is None else _f64(x0)
    x = np.empty(n)
    pol = policy if policy is not None else OraclePolicy()
    prm = Params(tol, maxit, replace_period, int(fallback), order, int(precond), int(stop_rule), int(rho_fp64),
                 int(emulate), int(vec16))
    res = Result()
    hist_rho = np.full(maxit + 1, np.nan)
    hist_act = np.zeros(max(maxit, 1), dtype=np.uint8)
    hist_flag = np.zeros(max(maxit, 1), dtype=np.uint8)
    rep_cap = maxit + 2
    rep_k = np.zeros(rep_cap, dtype=np.int32)
    rep_rho = np.zeros(rep_cap)
    h = Hist()
    h.hist_rho, h.hist_act, h.hist_flag = _p(hist_rho), _p(hist_act, C.c_uint8), _p(hist_flag, C.c_uint8)
    h.rep_k, h.rep_rho, h.rep_cap = _p(rep_k, C.c_int32), _p(rep_rho), rep_cap
    roll = None
    if roll_cap > 0:
        roll = dict(feat=np.zeros((roll_cap, 16), np.float32), next=np.zeros((roll_cap, 16), np.float32),
                    act=np.zeros(roll_cap, np.int32), rew=np.zeros(roll_cap, np.float32),
                    done=np.zeros(roll_cap, np.uint8))
        h.roll_cap = roll_cap
        h.roll_feat, h.roll_next = _p(roll["feat"], C.c_float), _p(roll["next"], C.c_float)
        h.roll_act, h.roll_rew = _p(roll["act"], C.c_int32), _p(roll["rew"], C.c_float)
        h.roll_done = _p(roll["done"], C.c_uint8)
    dumps = None
    if dump > 0:
        dumps = dict(alpha=np.full(dump, np.nan), beta=np.full(dump, np.nan),
                     p=np.zeros((dump, n)), r=np.zeros((dump, n)))
        h.dump_cap = dump
        h.hist_alpha, h.hist_beta = _p(dumps["alpha"]), _p(dumps["beta"])
        h.dump_p, h.dump_r = _p(dumps["p"]), _p(dumps["r"])
    lib().orc_cg(n, _p(_i32(A.row_ptr), C.c_int32), _p(_i32(A.col), C.c_int32), _p(_f64(A.val)),
                 _p(b), _p(x0), _p(x), C.byref(prm), C.byref(pol.s), C.byref(res), C.byref(h))
    k = res.iters
    nrep = min(res.n_replace, rep_cap)
    info = dict(status=res.status, iters=k, n_replace=res.n_replace, fallback_at=res.fallback_at,
                relres_true=res.relres_true, cost_sum=res.cost_sum,
                rho=hist_rho[:k + 1].copy(), actions=hist_act[:k].copy(), flags=hist_flag[:k].copy(),
                rep_k=rep_k[:nrep].copy(), rep_rho=rep_rho[:nrep].copy())
    if dumps is not None:
        info["dump"] = dumps
    if roll is not None:
        m = h.roll_n
        info["rollouts"] = {key: v[:m].copy() for key, v in roll.items()}
    return x, info


def cg_sr(A, b, action, x0=None, tol=1e-8, maxit=1000, replace_period=0, order=ORDER_PAIRWISE, dump=0):
    """Run the oracle's single-reduction CG (Chronopoulos-Gear: one SpMV and
    both inner products per iteration) with a fixed action.  dump > 0 keeps
    alpha, beta and the p, r, s used by the first `dump` iterations.
    Returns (x, info dict with histories)."""
    return _cg_variant("orc_cg_sr", A, b, action, x0, tol, maxit, replace_period, order, dump)


def cg_pipe(A, b, action, x0=None, tol=1e-8, maxit=1000, replace_period=0, order=ORDER_PAIRWISE, dump=0):
    """Run the oracle's pipelined CG (Ghysels-Vanroose: w = A r and z = A s by
    recurrence, the SpMV q = A w independent of the inner products) with a
    fixed action.  dump > 0 keeps alpha, beta and the p, r, s, w, z of the
    first `dump` iterations.  Returns (x, info dict with histories)."""
    return _cg_variant("orc_cg_pipe", A, b, action, x0, tol, maxit, replace_period, order, dump)


def _cg_variant(fn, A, b, action, x0, tol, maxit, replace_period, order, dump):
    n = A.n
    b = _f64(b)
    x0 = np.zeros(n) if x0 is None else _f64(x0)
    x = np.empty(n)
    prm = Params(tol, maxit, replace_period, 0, order, 0, 0, 0, 0, 0)
    res = Result()
    hist_rho = np.full(maxit + 1, np.nan)
    hist_act = np.zeros(max(maxit, 1), dtype=np.uint8)
    hist_flag = np.zeros(max(maxit, 1), dtype=np.uint8)
    rep_cap = maxit + 2
    rep_k = np.zeros(rep_cap, dtype=np.int32)
    rep_rho = np.zeros(rep_cap)
    h = Hist()
    h.hist_rho, h.hist_act, h.hist_flag = _p(hist_rho), _p(hist_act, C.c_uint8), _p(hist_flag, C.c_uint8)
    h.rep_k, h.rep_rho, h.rep_cap = _p(rep_k, C.c_int32), _p(rep_rho), rep_cap
    dumps = None
    if dump > 0:
        dumps = dict(alpha=np.full(dump, np.nan), beta=np.full(dump, np.nan),
                     p=np.zeros((dump, n)), r=np.zeros((dump, n)), s=np.zeros((dump, n)),
                     w=np.zeros((dump, n)), z=np.zeros((dump, n)))
        h.dump_cap = dump
        h.hist_alpha, h.hist_beta = _p(dumps["alpha"]), _p(dumps["beta"])
        h.dump_p, h.dump_r, h.dump_s = _p(dumps["p"]), _p(dumps["r"]), _p(dumps["s"])
        h.dump_w, h.dump_z = _p(dumps["w"]), _p(dumps["z"])
    rc = getattr(lib(), fn)(n, _p(_i32(A.row_ptr), C.c_int32), _p(_i32(A.col), C.c_int32), _p(_f64(A.val)),
                         _p(b), _p(x0), _p(x), int(action), C.byref(prm), C.byref(res), C.byref(h))
    if rc != 0:
        raise ValueError(f"the single-reduction and pipelined CG take actions 0..79, not {action}")
    k = res.iters
    nrep = min(res.n_replace, rep_cap)
    info = dict(status=res.status, iters=k, n_replace=res.n_replace, fallback_at=res.fallback_at,
                relres_true=res.relres_true, cost_sum=res.cost_sum,
                rho=hist_rho[:k + 1].copy(), actions=hist_act[:k].copy(), flags=hist_flag[:k].copy(),
                rep_k=rep_k[:nrep].copy(), rep_rho=rep_rho[:nrep].copy())
    if dumps is not None:
        info["dump"] = dumps
    return x, info


def cg_plain(A, b, tol=1e-8, maxit=1000):
    """Native fp64 CG without emulation (speed baseline).  Returns (x, iters, relres)."""
    x = np.zeros(A.n)
    it = C.c_int32(0)
    rr = C.c_double(0.0)
    lib().orc_cg_plain(A.n, _p(_i32(A.row_ptr), C.c_int32), _p(_i32(A.col), C.c_int32),
                       _p(_f64(A.val)), _p(_f64(b)), _p(x), tol, maxit, C.byref(it), C.byref(rr))
    return x, it.value, rr.value
