"""The allocation-free dot (mpcg_op_dot_noalloc) through the C ABI: its result
in device memory equals mpcg_op_dot's, bit for bit, in every format and vector
tier, on two calls in a row where the second has the smaller input (the static
partial array keeps the first call's contents), and both equal the oracle's
dot.  Sizes above the array's limit are refused before any launch."""
import ctypes as C

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_noalloc_dot_equals_op_dot_on_two_calls():
    import paper_2504_14268_amd as M

    L = M.lib()
    assert torch.cuda.is_available()
    rng = np.random.default_rng(21)
    mats = [M.Matrix(W.laplacian_2d(600)), M.Matrix(W.laplacian_2d(45))]   # n = 360000, then 2025
    assert mats[0].n > mats[1].n
    out = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    for fmt in range(4):
        for tier64 in (0, 1):
            for m in mats:                                    # larger call first, then the smaller one
                dt = np.float64 if tier64 else np.float32
                u = (rng.standard_normal(m.n) * 3).astype(dt)
                v = (rng.standard_normal(m.n) * 3).astype(dt)
                ud, vd = torch.from_numpy(u).cuda(), torch.from_numpy(v).cuda()
                want = C.c_double(0.0)
                rc = L.mpcg_op_dot(m.h, fmt, tier64, C.c_void_p(ud.data_ptr()), C.c_void_p(vd.data_ptr()),
                                   C.byref(want))
                assert rc == 0, L.mpcg_last_error()
                out.fill_(float("nan"))
                torch.cuda.synchronize()
                rc = L.mpcg_op_dot_noalloc(m.h, fmt, tier64, C.c_void_p(ud.data_ptr()), C.c_void_p(vd.data_ptr()),
                                           C.c_void_p(out.data_ptr()))
                assert rc == 0, L.mpcg_last_error()
                torch.cuda.synchronize()
                got = float(out.cpu()[0])
                assert got == want.value, (fmt, tier64, m.n, got, want.value)
                assert got == O.dot(u, v, fmt), (fmt, tier64, m.n)


def test_noalloc_dot_refuses_null_and_bad_format():
    import paper_2504_14268_amd as M

    L = M.lib()
    m = M.Matrix(W.laplacian_2d(8))
    x = torch.zeros(m.n, dtype=torch.float32, device="cuda")
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    p = C.c_void_p(x.data_ptr())
    assert L.mpcg_op_dot_noalloc(m.h, 4, 0, p, p, C.c_void_p(out.data_ptr())) == -1
    assert L.mpcg_op_dot_noalloc(m.h, 2, 0, p, p, None) == -1
    assert L.mpcg_op_dot_noalloc(None, 2, 0, p, p, C.c_void_p(out.data_ptr())) == -1
