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
    # never dereferenced: validation fails first; distinct 16 MiB-apart
    # addresses, so that only the argument under test is invalid
    fake = [ctypes.c_void_p(0x1000000 * (i + 1)) for i in range(6)]
    o = L.Opts()
    return L.tho_two_stage(dtype, n, k0, k, fake[0], ldv if ldv is not None else max(k0, 1),
                           fake[1], lda if lda is not None else max(k, 1),
                           fake[2], ldq if ldq is not None else max(k, 1), fake[3], max(k, 1),
                           fake[4], max(k, 1), ctypes.byref(o), fake[5], ws_bytes, None)


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


def _call_alias(n, k0, k, offs):
    """tho_two_stage with fake device pointers placed at byte offsets `offs`
    (V, A, Q, R, S) inside one imaginary buffer: validation rejects aliasing
    before any device work."""
    from paper_2602_14449_amd import _lib as L
    base = 0x10000000
    ptrs = [ctypes.c_void_p(base + o) for o in offs]
    o = L.Opts()
    # a NULL workspace (-16) is the first check after the alias check
    return L.tho_two_stage(0, n, k0, k, ptrs[0], k0, ptrs[1], k, ptrs[2], k, ptrs[3], k, ptrs[4], k,
                           ctypes.byref(o), None, 1 << 30, None)


def test_alias_detection():
    n, k0, k = 100, 8, 4
    mb = 1 << 20
    assert _call_alias(n, k0, k, [0, mb, 2 * mb, 3 * mb, 4 * mb]) == -16  # disjoint
    assert _call_alias(n, k0, k, [0, mb, mb, 3 * mb, 4 * mb]) == -9      # Q == A
    assert _call_alias(n, k0, k, [0, mb, 2 * mb, 0, 4 * mb]) == -11      # R inside V
    assert _call_alias(n, k0, k, [0, mb, 2 * mb, 3 * mb, 2 * mb + 8]) == -13  # S inside Q
    assert _call_alias(n, k0, k, [0, mb, 2 * mb, 3 * mb, 3 * mb + 24]) == -13  # S overlaps R


def test_blocks_side_by_side_are_not_aliases():
    # A and Q as two column slices of one wider row-major buffer (same ld)
    # share no element; a wrong (interval-only) check would reject them
    from paper_2602_14449_amd import _lib as L
    n, k0, k = 100, 8, 4
    base = 0x10000000
    o = L.Opts()
    ld = 2 * k
    args = lambda qoff: (0, n, k0, k, ctypes.c_void_p(base + (1 << 24)), k0,
                         ctypes.c_void_p(base), ld, ctypes.c_void_p(base + qoff), ld,
                         ctypes.c_void_p(base + (2 << 24)), k, ctypes.c_void_p(base + (3 << 24)), k,
                         ctypes.byref(o), None, 1 << 30, None)
    assert L.tho_two_stage(*args(8 * k)) == -16   # side by side: only the NULL workspace is reported
    assert L.tho_two_stage(*args(8 * (k - 1))) == -9  # shifted by one column less: overlap


def test_flag_and_choice_validation():
    from paper_2602_14449_amd import _lib as L
    import paper_2602_14449_amd as tho
    fake = ctypes.c_void_p(0x100000)
    o = L.Opts()
    o.flags = 4
    assert L.tho_two_stage(0, 100, 8, 4, fake, 8, fake, 4, fake, 4, fake, 4, fake, 4,
                           ctypes.byref(o), fake, 1 << 30, None) == -15
    o.flags = 0
    o.p_choice = 3
    assert L.tho_two_stage(0, 100, 8, 4, fake, 8, fake, 4, fake, 4, fake, 4, fake, 4,
                           ctypes.byref(o), fake, 1 << 30, None) == -15
    # workspace grows with the V-orthonormality check (Gram buffers) and with
    # the polar choice (Jacobi workspace), not with the finite check
    base = tho.workspace_bytes(1 << 16, 64, 32)
    assert tho.workspace_bytes(1 << 16, 64, 32, check_finite=True) == base
    assert tho.workspace_bytes(1 << 16, 64, 32, check_vorth=True) > base
    assert tho.workspace_bytes(1 << 16, 64, 32, p_choice="polar") > base
    info = ctypes.c_int32(7)
    assert L.tho_get_info(fake, None) == -2
