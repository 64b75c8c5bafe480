"""The C-ABI library loads and exports every function include/mpcg.h declares
(no compute call: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mpcg.h")
LIB = os.path.join(ROOT, "paper_2504_14268_amd", "libmpcg.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mpcg_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("mpcg_create_csr", "mpcg_set_policy", "mpcg_solve", "mpcg_destroy",
                 "mpcg_get_history", "mpcg_last_error"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmpcg.so not built")
def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(L, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmpcg.so not built")
def test_binding_covers_header():
    import paper_2504_14268_amd as M

    L = M.lib()
    for n in declared():
        fn = getattr(L, n)
        assert fn.restype in (ctypes.c_int, ctypes.c_char_p)
    assert L.mpcg_last_error() is not None


def test_binding_refuses_missing_library(tmp_path, monkeypatch):
    import paper_2504_14268_amd as M

    monkeypatch.setattr(M, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(M, "_lib", None)
    with pytest.raises(RuntimeError):
        M.lib()
