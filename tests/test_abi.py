"""C-ABI checks that need no GPU: the library loads, exports every symbol
declared in include/tho.h, and rejects invalid arguments (LAPACK-style -i
codes) before touching the device."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(tho_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


def test_exports_every_declared_symbol():
    from paper_2602_14449_amd import _lib
    syms = _declared_symbols()
    assert syms, "no declarations found"
    for s in syms:
        assert hasattr(_lib.lib, s), s


def test_version_and_strerror():
    from paper_2602_14449_amd import _lib
    assert _lib.tho_version().startswith(b"tho")
    assert _lib.tho_strerror(0) == b"success"
    assert _lib.tho_strerror(-100) == b"workspace too small"


def _call(n, k0, k, ldv=None, lda=None, ldq=None, ws_bytes=1 << 30, dtype=0):
    from paper_2602_14449_amd import _lib as L
    fake = ctypes.c_void_p(0x100000)  # never dereferenced: validation fails first
    o = L.Opts()
    return L.tho_two_stage(dtype, n, k0, k, fake, ldv if ldv is not None else max(k0, 1),
                           fake, lda if lda is not None else max(k, 1),
                           fake, ldq if ldq is not None else max(k, 1), fake, max(k, 1),
                           fake, max(k, 1), ctypes.byref(o), fake, ws_bytes, None)


@pytest.mark.parametrize("args,code", [
    ((10, 8, 4), -2),           # n < k0 + k
    ((100, -1, 4), -3),
    ((100, 200, 4), -3),        # k0 > THO_MAX_K0
    ((100, 8, 65), -4),         # k > THO_MAX_K
    ((100, 8, -2), -4),
])
def test_invalid_sizes(args, code):
    assert _call(*args) == code


def test_invalid_leading_dims():
    assert _call(100, 8, 4, ldv=7) == -6
    assert _call(100, 8, 4, lda=3) == -8
    assert _call(100, 8, 4, ldq=3) == -10


def test_bad_dtype_and_workspace():
    assert _call(100, 8, 4, dtype=5) == -1
    assert _call(100, 8, 4, ws_bytes=16) == -100


def test_workspace_query():
    import paper_2602_14449_amd as tho
    small = tho.workspace_bytes(4096, 16, 8)
    big = tho.workspace_bytes(1 << 22, 128, 64)
    assert 0 < small < big < (2 << 30)
    assert tho.workspace_bytes(100, 8, 0) == 0
