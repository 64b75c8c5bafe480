"""GPU parity of the hot-path kernels, one operation at a time, through the C
ABI: shadows, SpMV, dot, axpy and the fp64 residual must equal the oracle bit
for bit (same definitions, same summation trees)."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def M():
    import paper_2504_14268_amd as M

    M.lib()
    assert torch.cuda.is_available()
    return M


def dev(a, tier64):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64 if tier64 else np.float32)).cuda()


def eye(n):
    return W.CSR(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.ones(n))


def arrow_spd(n, seed):
    """Row 0 is dense (n entries): exercises SpMV rows spanning several LDS windows."""
    rng = np.random.default_rng(seed)
    rows, cols, vals = [], [], []
    off = rng.standard_normal(n - 1) * 0.1
    for j in range(1, n):
        rows += [0, j]
        cols += [j, 0]
        vals += [off[j - 1], off[j - 1]]
    rows += list(range(n))
    cols += list(range(n))
    d = np.full(n, 2.0)
    d[0] = np.abs(off).sum() + 1.0
    vals += list(d)
    A = W._from_coo(n, np.array(rows), np.array(cols), np.array(vals), "arrow")
    return A


MATS = {
    "lap3d_20": lambda: W.laplacian_3d(20),
    "rspd_5000": lambda: W.random_spd(5000, 3, spread=2.5),
    "band_3000": lambda: W.banded_spd(3000, 15, 4, spread=1.0),
    "arrow_9000": lambda: arrow_spd(9000, 5),
    "tiny_3": lambda: W.random_spd(3, 1, spread=0.0, tmin=1, tmax=1),
}


@pytest.mark.parametrize("name", list(MATS))
def test_shadows_bit_exact(M, name):
    A = MATS[name]()
    m = M.Matrix(A)
    f32, bf, hf, e = m.shadows()
    s32, sb, sh, oe = O.shadows(A)
    assert np.array_equal(f32.astype(np.float64), s32)
    assert np.array_equal((bf.astype(np.uint32) << 16).view(np.float32).astype(np.float64), sb)
    assert np.array_equal(hf.view(np.float16).astype(np.float64), sh)
    assert np.array_equal(e.astype(np.int32), oe)
    # q52: each byte is the high byte of the fp16 encoding of the same value
    q8 = m.shadow_q52()
    oq, oqe = O.shadow_q52(A)
    assert np.array_equal((q8.astype(np.uint16) << 8).view(np.float16).astype(np.float64), oq)
    assert np.array_equal(oqe, oe)
    # tf32: held in fp32 containers
    assert np.array_equal(m.shadow_tf32().astype(np.float64), O.shadow_tf32(A))


@pytest.mark.parametrize("name", list(MATS))
@pytest.mark.parametrize("fs", [0, 1, 2, 3, 4, 5])
@pytest.mark.parametrize("tier", [0, 1])
def test_spmv_bit_exact(M, name, fs, tier):
    A = MATS[name]()
    m = M.Matrix(A)
    rng = np.random.default_rng(fs * 2 + tier)
    p = rng.standard_normal(A.n) * 10.0 ** rng.uniform(-3, 3, A.n)
    p = p.astype(np.float32).astype(np.float64) if tier == 0 else p
    pd = dev(p, tier)
    qd = dev(np.zeros(A.n), tier)
    m.op_spmv(fs, tier, pd, qd)
    got = qd.cpu().numpy().astype(np.float64)
    want = O.spmv(A, p, fs, tier)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("n", [1, 7, 2048, 2049, 100003, 1 << 20])
@pytest.mark.parametrize("fd", [0, 1, 2, 3, 5])
@pytest.mark.parametrize("tier", [0, 1])
def test_dot_bit_exact(M, n, fd, tier):
    A = eye(n)                       # only the size matters here
    m = M.Matrix(A)
    rng = np.random.default_rng(n + fd)
    u = rng.standard_normal(A.n) * 3.0
    v = rng.standard_normal(A.n)
    if fd == 0:
        u[::97] *= 3e4          # some operands overflow fp16 -> inf is part of the definition
    if fd == 5:
        u[::89] *= 1e30         # far beyond fp16, inside tf32's (fp32's) range
        v[::83] *= 1e-40        # fp32 subnormals: tf32 keeps 2^-136 steps
    if tier == 0:
        u, v = u.astype(np.float32).astype(np.float64), v.astype(np.float32).astype(np.float64)
    got = m.op_dot(fd, tier, dev(u, tier), dev(v, tier))
    want = O.dot(u, v, fd)
    assert got == want or (np.isnan(got) and np.isnan(want))


@pytest.mark.parametrize("fa", [0, 1, 2, 3, 5])
def test_axpy_bit_exact(M, fa):
    n = 10007
    A = eye(n)
    m = M.Matrix(A)
    tier = 1 if fa == 3 else 0
    rng = np.random.default_rng(fa)
    u = rng.standard_normal(n) * 10.0 ** rng.uniform(-6, 5, n)
    y = rng.standard_normal(n) * 10.0 ** rng.uniform(-6, 5, n)
    if tier == 0:
        u, y = u.astype(np.float32).astype(np.float64), y.astype(np.float32).astype(np.float64)
    yd = dev(y, tier)
    alpha = -0.7310585786300049
    m.op_axpy(fa, alpha, dev(u, tier), yd)
    assert np.array_equal(yd.cpu().numpy().astype(np.float64), O.axpy(alpha, u, y, fa))


@pytest.mark.parametrize("name", ["lap3d_20", "rspd_5000", "arrow_9000"])
def test_residual_bit_exact(M, name):
    A = MATS[name]()
    m = M.Matrix(A)
    rng = np.random.default_rng(2)
    b, x = rng.standard_normal(A.n), rng.standard_normal(A.n)
    r = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    m.op_residual(dev(b, 1), dev(x, 1), r)
    assert np.array_equal(r.cpu().numpy(), O.residual(A, b, x))


def test_policy_decisions_bit_exact(M):
    """Identical states give identical state indices and actions (Q-table and MLP)."""
    rng = np.random.default_rng(9)
    m = 4000
    k = rng.integers(0, 3000, m)
    rho = 10.0 ** rng.uniform(-17, 1, m)
    edges = O.residual_edges()
    rho[:9] = edges                      # exact bin edges, and both neighbouring doubles
    rho[9:18] = np.nextafter(edges, 1.0)
    rho[18:27] = np.nextafter(edges, 0.0)
    stag = rng.integers(0, 2, m)
    q = rng.standard_normal((100, 64))
    q[:, 5] = q[:, 9] = 10.0             # ties: the lowest index wins
    P = M.Policy(kind=M.POLICY_QTABLE)
    P.set_qtable(q)
    st, ac = P.decide(k, rho, stag)
    op = O.OraclePolicy(kind=O.POL_QTABLE, q=q)
    want_s = np.array([op.state(int(k[i]), float(rho[i]), int(stag[i])) for i in range(m)])
    assert np.array_equal(st, want_s)
    assert np.array_equal(ac, np.argmax(q[want_s], axis=1))
    assert np.all(ac[np.max(q[want_s], axis=1) == 10.0] == 5)
    # another bin layout: the library derives its thresholds from b_res and
    # eps_min; the oracle from its own decimal computation
    e6 = O.residual_edges(7, 12)
    rho2 = rho.copy()
    rho2[:6], rho2[6:12], rho2[12:18] = e6, np.nextafter(e6, 1.0), np.nextafter(e6, 0.0)
    q6 = rng.standard_normal((7 * 3 * 2, 64))
    P6 = M.Policy(kind=M.POLICY_QTABLE, b_res=7, eps_min=1e-12, b_it=3, t_bin=900)
    P6.set_qtable(q6)
    st6, ac6 = P6.decide(k, rho2, stag)
    op6 = O.OraclePolicy(kind=O.POL_QTABLE, q=q6, b_res=7, eps_min=1e-12, b_it=3, t_bin=900)
    want6 = np.array([op6.state(int(k[i]), float(rho2[i]), int(stag[i])) for i in range(m)])
    assert np.array_equal(st6, want6)
    assert np.array_equal(ac6, np.argmax(q6[want6], axis=1))
    # MLP: logits from the fp32 fixed-order decision path
    from test_oracle_policy import mlp_weights

    w = mlp_weights(3)
    P2 = M.Policy(kind=M.POLICY_MLP)
    P2.set_mlp(w)
    feat = (rng.standard_normal((500, 16)) * 4).astype(np.float32)
    st2, ac2 = P2.decide(k[:500], rho[:500], stag[:500], feat)
    op2 = O.OraclePolicy(kind=O.POL_MLP, mlp=w)
    want = np.array([int(np.argmax(op2.mlp_logits(f))) for f in feat])
    assert np.array_equal(ac2, want)
