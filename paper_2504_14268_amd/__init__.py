"""Python binding of libmpcg.so (include/mpcg.h): argument marshalling only.

Every step of the solver runs in the HIP kernels of the library; torch supplies
device memory and the stream.  Importing this package does not need a GPU; any
call that reaches the library raises if libmpcg.so has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmpcg.so")

FP16, BF16, FP32, FP64, Q52, TF32 = 0, 1, 2, 3, 4, 5
FORMATS = {"fp16": FP16, "bf16": BF16, "fp32": FP32, "fp64": FP64, "q52": Q52, "tf32": TF32}
POLICY_FIXED, POLICY_QTABLE, POLICY_QTABLE_TRAIN, POLICY_MLP = 0, 1, 2, 3
CONVERGED, MAXIT, CONVERGED_FALLBACK, BREAKDOWN = 0, 1, 2, 3
FLAG_REPLACED, FLAG_EXPLORED, FLAG_FALLBACK, FLAG_SWITCH = 1, 2, 4, 8
# c(fp16), c(bf16), c(fp32), c(fp64), c(tf32)
COSTS = {"C1": (0.8, 0.6, 1.0, 2.0, 0.8), "C2": (0.5, 0.4, 1.5, 3.0, 0.5)}


def action(f_spmv: int, f_dot: int, f_axpy: int) -> int:
    """The library's action code of a format triple (mpcg_action)."""
    a = lib().mpcg_action(f_spmv, f_dot, f_axpy)
    if a < 0:
        _check(a, "mpcg_action")
    return a


def decode(a: int):
    """(f_spmv, f_dot, f_axpy) of an action code, as the library reads it."""
    fs, fd, fa = C.c_int32(), C.c_int32(), C.c_int32()
    _check(lib().mpcg_action_formats(int(a), C.byref(fs), C.byref(fd), C.byref(fa)), "action_formats")
    return fs.value, fd.value, fa.value


class PolicyDesc(C.Structure):
    _fields_ = [
        ("kind", C.c_int32), ("fixed_action", C.c_int32), ("t_bin", C.c_int32),
        ("b_it", C.c_int32), ("b_res", C.c_int32), ("w_stag", C.c_int32),
        ("lr", C.c_double), ("gamma", C.c_double),
        ("w1", C.c_double), ("w2", C.c_double), ("w3", C.c_double), ("eps_min", C.c_double),
        ("cost", C.c_double * 4), ("seed", C.c_uint64),
        ("replace_period", C.c_int32), ("decision_period", C.c_int32),
        ("per_op", C.c_int32), ("nfmt", C.c_int32), ("cost_tf32", C.c_double),
    ]


class SolveOpts(C.Structure):
    _fields_ = [("replace_period", C.c_int32), ("fallback", C.c_int32),
                ("chunk", C.c_int32), ("profile", C.c_int32),
                ("spmv_rows", C.c_int32), ("index16", C.c_int32),
                ("precond", C.c_int32), ("stop_rule", C.c_int32),
                ("rho_fp64", C.c_int32), ("emulate", C.c_int32),
                ("vec16", C.c_int32), ("variant", C.c_int32)]


class Profile(C.Structure):
    _fields_ = [("n_iter_slots", C.c_int32), ("n_resid_slots", C.c_int32),
                ("n_idle_slots", C.c_int32), ("reserved", C.c_int32),
                ("ka_iter_ms", C.c_double), ("kb_iter_ms", C.c_double), ("kx_iter_ms", C.c_double),
                ("ks_iter_ms", C.c_double),
                ("resid_ms", C.c_double), ("idle_ms", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


class MatrixInfo(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("index16", C.c_int32), ("reserved", C.c_int32)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("n_replace", C.c_int32),
                ("fallback_at", C.c_int32), ("relres_true", C.c_double), ("cost_sum", C.c_double),
                ("time_ms", C.c_double), ("slots", C.c_int32), ("spmv_rows", C.c_int32),
                ("index16", C.c_int32), ("reserved", C.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


class BatchOpts(C.Structure):
    _fields_ = [("workgroups", C.c_int32), ("spmv_rows", C.c_int32), ("order", C.c_int32),
                ("autotune_iters", C.c_int32), ("split_rows", C.c_int32), ("strategy", C.c_int32)]


class BatchInfo(C.Structure):
    _fields_ = [("time_ms", C.c_double), ("tune_ms", C.c_double), ("workgroups", C.c_int32),
                ("spmv_rows", C.c_int32), ("tuned", C.c_int32), ("split_rows", C.c_int32),
                ("n_split", C.c_int32), ("strategy", C.c_int32), ("persistent_ms", C.c_double),
                ("split_ms", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


class MlpTrainDesc(C.Structure):
    _fields_ = [("batch", C.c_int32), ("epochs", C.c_int32), ("lr", C.c_double), ("beta1", C.c_double),
                ("beta2", C.c_double), ("eps", C.c_double), ("gamma", C.c_double)]


class TrainDesc(C.Structure):
    _fields_ = [("episodes", C.c_int32), ("maxit", C.c_int32), ("tol", C.c_double),
                ("eps_start", C.c_double), ("eps_end", C.c_double), ("order", C.c_int32),
                ("first_episode", C.c_int32), ("total_episodes", C.c_int32), ("reserved", C.c_int32)]


class EpisodeResult(C.Structure):
    _fields_ = [("system", C.c_int32), ("episode", C.c_int32), ("epsilon", C.c_double), ("res", Result)]

    def as_dict(self):
        return {"system": self.system, "episode": self.episode, "epsilon": self.epsilon, **self.res.as_dict()}


_lib = None


def lib():
    """The loaded library; raises if it has not been built (no fallback path exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libmpcg.so not built at {LIB_PATH}: run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        L.mpcg_last_error.restype = C.c_char_p
        sig = {
            "mpcg_create_csr": [i64, i64, vp, vp, vp, C.c_int, vp, C.POINTER(vp)],
            "mpcg_destroy": [vp],
            "mpcg_get_info": [vp, C.POINTER(MatrixInfo)],
            "mpcg_get_shadows": [vp, vp, vp, vp, vp],
            "mpcg_get_shadow_q52": [vp, vp],
            "mpcg_get_shadow_tf32": [vp, vp],
            "mpcg_action": [C.c_int, C.c_int, C.c_int],
            "mpcg_action_formats": [C.c_int, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)],
            "mpcg_get_precond": [vp, vp],
            "mpcg_residual_thresholds": [i32, d, vp],
            "mpcg_policy_create": [C.POINTER(PolicyDesc), C.POINTER(vp)],
            "mpcg_policy_destroy": [vp],
            "mpcg_policy_set_qtable": [vp, vp],
            "mpcg_policy_get_qtable": [vp, vp],
            "mpcg_policy_set_episode": [vp, i64, d],
            "mpcg_policy_set_mlp": [vp, vp, vp, vp, vp, vp, vp],
            "mpcg_policy_rollouts_enable": [vp, i32],
            "mpcg_policy_rollouts_count": [vp, C.POINTER(i32)],
            "mpcg_policy_rollouts_reset": [vp],
            "mpcg_policy_get_rollouts": [vp, vp, vp, vp, vp, vp, i32, C.POINTER(i32)],
            "mpcg_policy_decide": [vp, i32, vp, vp, vp, vp, vp, vp],
            "mpcg_set_policy": [vp, vp],
            "mpcg_set_options": [vp, C.POINTER(SolveOpts)],
            "mpcg_solve": [vp, vp, vp, d, i32, C.POINTER(Result)],
            "mpcg_get_history": [vp, vp, vp, vp, i32, vp, vp, i32, C.POINTER(i32)],
            "mpcg_op_spmv": [vp, C.c_int, C.c_int, vp, vp],
            "mpcg_op_dot": [vp, C.c_int, C.c_int, vp, vp, C.POINTER(d)],
            "mpcg_op_dot_noalloc": [vp, C.c_int, C.c_int, vp, vp, vp],
            "mpcg_gather_floor": [vp, vp, i32, C.POINTER(d)],
            "mpcg_op_axpy": [vp, C.c_int, d, vp, vp],
            "mpcg_op_residual": [vp, vp, vp, vp],
            "mpcg_get_profile": [vp, C.POINTER(Profile)],
            "mpcg_train_qlearning": [vp, i32, vp, vp, vp, C.POINTER(TrainDesc), vp],
            "mpcg_solve_batched": [i32, vp, vp, vp, vp, vp, C.POINTER(BatchOpts), vp, C.POINTER(BatchInfo)],
            "mpcg_mlp_create": [vp, vp, C.POINTER(vp)],
            "mpcg_mlp_destroy": [vp],
            "mpcg_mlp_set_params": [vp, vp],
            "mpcg_mlp_get_params": [vp, vp],
            "mpcg_mlp_forward": [vp, vp, i32, vp],
            "mpcg_mlp_grad": [vp, vp, vp, vp, i32, vp, C.POINTER(C.c_float)],
            "mpcg_mlp_train": [vp, vp, vp, vp, vp, vp, i32, C.POINTER(MlpTrainDesc), vp],
            "mpcg_policy_set_mlp_from": [vp, vp],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = C.c_int
        _lib = L
    return _lib


class MPCGError(RuntimeError):
    pass


def _check(rc: int, what: str):
    if rc != 0:
        msg = lib().mpcg_last_error().decode(errors="replace")
        raise MPCGError(f"{what} failed ({rc}): {msg}")


def _np_ptr(a: np.ndarray):
    return C.c_void_p(a.ctypes.data)


def _t_ptr(t):
    return C.c_void_p(t.data_ptr())


def _stream_handle(stream):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def residual_thresholds(b_res: int = 10, eps_min: float = 1e-16):
    """The library's residual-bin thresholds T_1..T_{b_res-1} (mpcg_residual_thresholds)."""
    out = np.zeros(max(b_res - 1, 1))
    _check(lib().mpcg_residual_thresholds(b_res, eps_min, _np_ptr(out)), "mpcg_residual_thresholds")
    return out[:b_res - 1]


class Policy:
    """A precision policy (fixed, Q-table greedy, Q-table training, MLP)."""

    def __init__(self, kind=POLICY_FIXED, fixed_action=63, t_bin=1000, b_it=5, b_res=10, w_stag=10,
                 lr=0.1, gamma=0.9, w=(1.0, 0.1, 10.0), eps_min=1e-16, cost="C1", seed=0,
                 replace_period=50, decision_period=1, per_op=0, nfmt=4):
        d = PolicyDesc()
        d.kind, d.fixed_action, d.t_bin, d.b_it, d.b_res, d.w_stag = kind, fixed_action, t_bin, b_it, b_res, w_stag
        d.lr, d.gamma = lr, gamma
        d.w1, d.w2, d.w3 = w
        d.eps_min = eps_min
        costs = COSTS[cost] if isinstance(cost, str) else cost
        for i in range(4):
            d.cost[i] = costs[i]
        d.cost_tf32 = costs[4] if len(costs) > 4 else costs[0]
        d.nfmt = int(nfmt)
        d.seed = seed
        d.replace_period = replace_period
        d.decision_period = decision_period
        d.per_op = int(per_op)
        self.desc = d
        self.n_states = b_res * b_it * 2
        h = C.c_void_p()
        _check(lib().mpcg_policy_create(C.byref(d), C.byref(h)), "mpcg_policy_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None) and _lib is not None:
            lib().mpcg_policy_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_qtable(self, q):
        q = np.ascontiguousarray(q, dtype=np.float64).reshape(self.n_states, 64)
        _check(lib().mpcg_policy_set_qtable(self.h, _np_ptr(q)), "set_qtable")

    def qtable(self):
        q = np.empty((self.n_states, 64))
        _check(lib().mpcg_policy_get_qtable(self.h, _np_ptr(q)), "get_qtable")
        return q

    def set_episode(self, episode: int, epsilon: float):
        _check(lib().mpcg_policy_set_episode(self.h, episode, epsilon), "set_episode")

    def set_mlp(self, w: dict):
        arrs = [np.ascontiguousarray(w[k], dtype=np.float32) for k in ("W1", "b1", "W2", "b2", "W3", "b3")]
        self._mlp_keep = arrs
        _check(lib().mpcg_policy_set_mlp(self.h, *[_np_ptr(a) for a in arrs]), "set_mlp")

    def rollouts_enable(self, capacity: int):
        _check(lib().mpcg_policy_rollouts_enable(self.h, capacity), "rollouts_enable")

    def rollouts_reset(self):
        _check(lib().mpcg_policy_rollouts_reset(self.h), "rollouts_reset")

    def rollouts(self, cap: int | None = None):
        n = C.c_int32(0)
        _check(lib().mpcg_policy_rollouts_count(self.h, C.byref(n)), "rollouts_count")
        m = n.value if cap is None else min(cap, n.value)
        out = dict(feat=np.zeros((m, 16), np.float32), next=np.zeros((m, 16), np.float32),
                   act=np.zeros(m, np.int32), rew=np.zeros(m, np.float32), done=np.zeros(m, np.uint8))
        if m:
            got = C.c_int32(0)
            _check(lib().mpcg_policy_get_rollouts(self.h, _np_ptr(out["feat"]), _np_ptr(out["next"]),
                                                  _np_ptr(out["act"]), _np_ptr(out["rew"]),
                                                  _np_ptr(out["done"]), m, C.byref(got)), "get_rollouts")
        return out

    def decide(self, k, rho, stag, feat=None):
        k = np.ascontiguousarray(k, dtype=np.int64)
        rho = np.ascontiguousarray(rho, dtype=np.float64)
        stag = np.ascontiguousarray(stag, dtype=np.int32)
        m = k.size
        st = np.zeros(m, np.int32)
        ac = np.zeros(m, np.int32)
        fp = None
        if feat is not None:
            feat = np.ascontiguousarray(feat, dtype=np.float32).reshape(m, 16)
            fp = _np_ptr(feat)
        _check(lib().mpcg_policy_decide(self.h, m, _np_ptr(k), _np_ptr(rho), _np_ptr(stag), fp,
                                        _np_ptr(st), _np_ptr(ac)), "policy_decide")
        return st, ac


MLP_PARAMS = 128 * 16 + 128 + 128 * 128 + 128 + 64 * 128 + 64
MLP_SHAPES = (("W1", (128, 16)), ("b1", (128,)), ("W2", (128, 128)), ("b2", (128,)), ("W3", (64, 128)), ("b3", (64,)))


def mlp_pack(w: dict) -> np.ndarray:
    """Parameter dict -> float32[26944] in the order W1 | b1 | W2 | b2 | W3 | b3."""
    return np.concatenate([np.asarray(w[k], dtype=np.float32).reshape(-1) for k, _ in MLP_SHAPES])


def mlp_unpack(v) -> dict:
    out, o = {}, 0
    for k, shp in MLP_SHAPES:
        size = int(np.prod(shp))
        out[k] = np.asarray(v[o:o + size], dtype=np.float32).reshape(shp)
        o += size
    return out


def mlp_init_params(seed: int) -> dict:
    """Seeded He-normal weights (float32), zero biases."""
    rng = np.random.default_rng(seed)
    return dict(W1=(rng.standard_normal((128, 16)) * np.sqrt(2.0 / 16)).astype(np.float32),
                b1=np.zeros(128, np.float32),
                W2=(rng.standard_normal((128, 128)) * np.sqrt(2.0 / 128)).astype(np.float32),
                b2=np.zeros(128, np.float32),
                W3=(rng.standard_normal((64, 128)) * np.sqrt(1.0 / 128)).astype(np.float32),
                b3=np.zeros(64, np.float32))


class Mlp:
    """The MLP policy network with its Adam trainer (mpcg_mlp_*)."""

    def __init__(self, params: dict, stream=None):
        v = np.ascontiguousarray(mlp_pack(params))
        h = C.c_void_p()
        _check(lib().mpcg_mlp_create(_np_ptr(v), _stream_handle(stream), C.byref(h)), "mpcg_mlp_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None) and _lib is not None:
            lib().mpcg_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params: dict):
        v = np.ascontiguousarray(mlp_pack(params))
        _check(lib().mpcg_mlp_set_params(self.h, _np_ptr(v)), "mlp_set_params")

    def params(self) -> dict:
        v = np.empty(MLP_PARAMS, dtype=np.float32)
        _check(lib().mpcg_mlp_get_params(self.h, _np_ptr(v)), "mlp_get_params")
        return mlp_unpack(v)

    def forward(self, feat):
        """feat: float32 device tensor [n, 16] -> logits float32 device tensor [n, 64]."""
        import torch

        assert feat.is_cuda and feat.dtype == torch.float32 and feat.is_contiguous() and feat.shape[1] == 16
        out = torch.empty((feat.shape[0], 64), dtype=torch.float32, device=feat.device)
        _check(lib().mpcg_mlp_forward(self.h, _t_ptr(feat), feat.shape[0], _t_ptr(out)), "mlp_forward")
        return out

    def grad(self, feat, act, target):
        """One batch's gradient (device tensors) -> (dict of float32 arrays, loss)."""
        g = np.empty(MLP_PARAMS, dtype=np.float32)
        loss = C.c_float()
        _check(lib().mpcg_mlp_grad(self.h, _t_ptr(feat), _t_ptr(act), _t_ptr(target), feat.shape[0], _np_ptr(g),
                                   C.byref(loss)), "mlp_grad")
        return mlp_unpack(g), loss.value

    def train(self, data: dict, batch=256, epochs=1, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, gamma=0.9):
        """data: device tensors feat, next (float32 [n,16]), act (int32), rew (float32), done (uint8)."""
        n = int(data["act"].shape[0])
        for k in ("feat", "next", "act", "rew", "done"):
            assert data[k].is_cuda and data[k].is_contiguous() and data[k].shape[0] == n
        d = MlpTrainDesc(batch, epochs, lr, beta1, beta2, eps, gamma)
        out = np.zeros(max(epochs, 1), dtype=np.float32)
        _check(lib().mpcg_mlp_train(self.h, _t_ptr(data["feat"]), _t_ptr(data["next"]), _t_ptr(data["act"]),
                                    _t_ptr(data["rew"]), _t_ptr(data["done"]), n, C.byref(d), _np_ptr(out)),
               "mlp_train")
        return out[:epochs]

    def to_policy(self, policy: "Policy"):
        _check(lib().mpcg_policy_set_mlp_from(policy.h, self.h), "policy_set_mlp_from")


def solve_batched(systems, tol=1e-8, maxit=1000, workgroups=0, spmv_rows=0, order=0, autotune_iters=0,
                  split_rows=0, strategy=0):
    """One persistent launch over systems = [(Matrix, b, x), ...] (device float64
    tensors; x holds x0 and receives the solution).  tol / maxit: scalars or
    per-system lists.  Returns (list of result dicts, batch info dict)."""
    m = len(systems)
    tols = np.ascontiguousarray(np.broadcast_to(np.asarray(tol, dtype=np.float64), (m,)))
    mits = np.ascontiguousarray(np.broadcast_to(np.asarray(maxit, dtype=np.int32), (m,)))
    for s in systems:
        assert s[1].is_cuda and s[2].is_cuda and s[1].numel() == s[0].n and s[2].numel() == s[0].n
        assert s[1].dtype == s[2].dtype and s[1].element_size() == 8 and s[1].is_contiguous() and s[2].is_contiguous()
    hs = (C.c_void_p * max(m, 1))(*[s[0].h for s in systems])
    bs = (C.c_void_p * max(m, 1))(*[s[1].data_ptr() for s in systems])
    xs = (C.c_void_p * max(m, 1))(*[s[2].data_ptr() for s in systems])
    res = (Result * max(m, 1))()
    info = BatchInfo()
    o = BatchOpts(workgroups, spmv_rows, order, autotune_iters, split_rows, strategy)
    _check(lib().mpcg_solve_batched(m, hs, bs, xs, _np_ptr(tols), _np_ptr(mits), C.byref(o), res, C.byref(info)),
           "mpcg_solve_batched")
    return [res[i].as_dict() for i in range(m)], info.as_dict()


def train_qlearning(policy: "Policy", systems, episodes=5, maxit=1000, tol=1e-8, eps_start=1.0, eps_end=0.1,
                    order=0, first_episode=1, total_episodes=0):
    """Tabular Q-learning over `systems` = [(Matrix, b, x), ...] (b, x float64 device
    tensors; x is overwritten).  Returns one dict per episode (mpcg_train_qlearning)."""
    m = len(systems)
    hs = (C.c_void_p * max(m, 1))(*[s[0].h for s in systems])
    bs = (C.c_void_p * max(m, 1))(*[s[1].data_ptr() for s in systems])
    xs = (C.c_void_p * max(m, 1))(*[s[2].data_ptr() for s in systems])
    for s in systems:
        assert s[1].is_cuda and s[2].is_cuda and s[1].numel() == s[0].n and s[2].numel() == s[0].n
    d = TrainDesc(episodes, maxit, tol, eps_start, eps_end, order, first_episode, total_episodes, 0)
    out = (EpisodeResult * max(m * episodes, 1))()
    _check(lib().mpcg_train_qlearning(policy.h, m, hs, bs, xs, C.byref(d), out), "mpcg_train_qlearning")
    return [out[j].as_dict() for j in range(m * episodes)]


class Matrix:
    """A CSR matrix on the device with its shadows; solves run on `stream`."""

    def __init__(self, A, stream=None):
        rp = np.ascontiguousarray(A.row_ptr, dtype=np.int32)
        ci = np.ascontiguousarray(A.col, dtype=np.int32)
        v = np.ascontiguousarray(A.val, dtype=np.float64)
        self.n, self.nnz = int(A.n), int(rp[-1])
        self._stream = stream
        h = C.c_void_p()
        _check(lib().mpcg_create_csr(self.n, self.nnz, _np_ptr(rp), _np_ptr(ci), _np_ptr(v), 0,
                                     _stream_handle(stream), C.byref(h)), "mpcg_create_csr")
        self.h = h
        self.policy = None

    @classmethod
    def from_device(cls, row_ptr, col, val, stream=None) -> "Matrix":
        """A CSR matrix whose arrays are already on the device: torch tensors
        (int32 row_ptr[n+1], int32 col[nnz], float64 val[nnz], contiguous)."""
        for t, dt in ((row_ptr, "torch.int32"), (col, "torch.int32"), (val, "torch.float64")):
            assert t.is_cuda and t.is_contiguous() and str(t.dtype) == dt, "device CSR arrays of the stated types"
        self = cls.__new__(cls)
        self.n = int(row_ptr.numel()) - 1
        self.nnz = int(col.numel())
        self._stream = stream
        h = C.c_void_p()
        _check(lib().mpcg_create_csr(self.n, self.nnz, _t_ptr(row_ptr), _t_ptr(col), _t_ptr(val), 1,
                                     _stream_handle(stream), C.byref(h)), "mpcg_create_csr")
        self.h = h
        self.policy = None
        return self

    def close(self):
        if getattr(self, "h", None) and _lib is not None:
            lib().mpcg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        i = MatrixInfo()
        _check(lib().mpcg_get_info(self.h, C.byref(i)), "get_info")
        return {"n": i.n, "nnz": i.nnz, "index16": bool(i.index16)}

    def set_policy(self, policy: Policy | None):
        _check(lib().mpcg_set_policy(self.h, policy.h if policy is not None else None), "set_policy")
        self.policy = policy

    def set_options(self, replace_period=50, fallback=False, chunk=0, profile=False, spmv_rows=0, index16=0,
                    precond=0, stop_rule=0, rho_fp64=0, emulate=0, vec16=0, variant=0):
        """variant 1: single-reduction CG (Chronopoulos-Gear); 2: pipelined CG
        (Ghysels-Vanroose); both two launches per iteration, fixed actions."""
        o = SolveOpts(replace_period, int(fallback), chunk, int(profile), spmv_rows, index16, int(precond),
                      int(stop_rule), int(rho_fp64), int(emulate), int(vec16), int(variant))
        _check(lib().mpcg_set_options(self.h, C.byref(o)), "set_options")

    def solve(self, b, x, tol=1e-8, maxit=1000) -> dict:
        """b, x: float64 device tensors of length n; x is the initial guess and the result."""
        assert b.dtype.is_floating_point and b.element_size() == 8 and b.is_contiguous() and b.numel() == self.n
        assert x.dtype == b.dtype and x.is_contiguous() and x.numel() == self.n and x.is_cuda and b.is_cuda
        r = Result()
        _check(lib().mpcg_solve(self.h, _t_ptr(b), _t_ptr(x), tol, maxit, C.byref(r)), "mpcg_solve")
        return r.as_dict()

    def profile(self) -> dict:
        pr = Profile()
        _check(lib().mpcg_get_profile(self.h, C.byref(pr)), "get_profile")
        return pr.as_dict()

    def history(self, cap: int | None = None):
        n = C.c_int32(0)
        _check(lib().mpcg_get_history(self.h, None, None, None, 0, None, None, 0, C.byref(n)), "history")
        k1 = n.value
        cap = k1 if cap is None else cap
        rho = np.zeros(k1)
        act = np.zeros(max(k1 - 1, 1), np.uint8)
        flg = np.zeros(max(k1 - 1, 1), np.uint8)
        rep_k = np.zeros(k1 + 1, np.int32)
        rep_rho = np.zeros(k1 + 1)
        _check(lib().mpcg_get_history(self.h, _np_ptr(rho), _np_ptr(act), _np_ptr(flg), k1,
                                      _np_ptr(rep_k), _np_ptr(rep_rho), k1 + 1, C.byref(n)), "history")
        return dict(rho=rho, actions=act[:k1 - 1], flags=flg[:k1 - 1], rep_k=rep_k, rep_rho=rep_rho)

    def shadows(self):
        f32 = np.zeros(self.nnz, np.float32)
        bf = np.zeros(self.nnz, np.uint16)
        hf = np.zeros(self.nnz, np.uint16)
        e = np.zeros(self.n, np.int8)
        _check(lib().mpcg_get_shadows(self.h, _np_ptr(f32), _np_ptr(bf), _np_ptr(hf), _np_ptr(e)), "shadows")
        return f32, bf, hf, e

    def precond_inverse(self):
        out = np.zeros(self.n, np.float32)
        _check(lib().mpcg_get_precond(self.h, _np_ptr(out)), "get_precond")
        return out

    def shadow_tf32(self):
        out = np.zeros(self.nnz, np.float32)
        _check(lib().mpcg_get_shadow_tf32(self.h, _np_ptr(out)), "shadow_tf32")
        return out

    def shadow_q52(self):
        out = np.zeros(self.nnz, np.uint8)
        _check(lib().mpcg_get_shadow_q52(self.h, _np_ptr(out)), "shadow_q52")
        return out

    def op_spmv(self, fmt, tier64, p, q):
        _check(lib().mpcg_op_spmv(self.h, fmt, tier64, _t_ptr(p), _t_ptr(q)), "op_spmv")

    def op_dot(self, fmt, tier64, u, v) -> float:
        out = C.c_double(0.0)
        _check(lib().mpcg_op_dot(self.h, fmt, tier64, _t_ptr(u), _t_ptr(v), C.byref(out)), "op_dot")
        return out.value

    def op_dot_noalloc(self, fmt, tier64, u, v, out):
        """dot_f(u, v) into the device double out[0], with no allocation (mpcg_op_dot_noalloc)."""
        _check(lib().mpcg_op_dot_noalloc(self.h, fmt, tier64, _t_ptr(u), _t_ptr(v), _t_ptr(out)), "op_dot_noalloc")

    def gather_floor(self, p, repeats=20) -> float:
        """Mean microseconds of the flat-gather floor kernel over this matrix's columns."""
        us = C.c_double(0.0)
        _check(lib().mpcg_gather_floor(self.h, _t_ptr(p), repeats, C.byref(us)), "gather_floor")
        return us.value

    def op_axpy(self, fmt, alpha, u, y):
        _check(lib().mpcg_op_axpy(self.h, fmt, alpha, _t_ptr(u), _t_ptr(y)), "op_axpy")

    def op_residual(self, b, x, r):
        _check(lib().mpcg_op_residual(self.h, _t_ptr(b), _t_ptr(x), _t_ptr(r)), "op_residual")
