"""tho_two_stage_noalloc (library-owned static scratch, no device allocation)
against tho_two_stage with a caller workspace, both called through the C ABI
on the same inputs.  Both run the same kernels in the same order, so the
outputs must agree bit for bit.  Two calls in a row, the second with a
smaller problem, so that the second call runs on scratch that still holds the
first call's data; a complex call and the size limit are checked too."""

import ctypes

import numpy as np
import pytest
import torch

import tho_workloads as W
from gpu_util import require_gpu, to_dev, to_host

pytestmark = pytest.mark.gpu


def _bufs(n, k0, k, dtype):
    dev = torch.device("cuda")
    return (torch.full((n, k), float("nan"), dtype=dtype, device=dev),
            torch.full((k, k), float("nan"), dtype=dtype, device=dev),
            torch.full((max(k0, 1), k), float("nan"), dtype=dtype, device=dev))


def _with_workspace(L, code, V, A, n, k0, k):
    Q, R, S = _bufs(n, k0, k, A.dtype)
    o = L.Opts()
    nb = L.c_sz(0)
    L.check(L.tho_two_stage_workspace(code, n, k0, k, ctypes.byref(o), ctypes.byref(nb)), "workspace")
    ws = torch.empty(max(nb.value, 1), dtype=torch.uint8, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    rc = L.tho_two_stage(code, n, k0, k, V.data_ptr(), k0, A.data_ptr(), k, Q.data_ptr(), k,
                         R.data_ptr(), k, S.data_ptr(), k, ctypes.byref(o), ws.data_ptr(), ws.numel(), st)
    L.check(rc, "tho_two_stage")
    torch.cuda.synchronize()
    return to_host(Q), to_host(R), to_host(S)


def _noalloc(L, code, V, A, n, k0, k):
    Q, R, S = _bufs(n, k0, k, A.dtype)
    o = L.Opts()
    st = torch.cuda.current_stream().cuda_stream
    rc = L.tho_two_stage_noalloc(code, n, k0, k, V.data_ptr(), k0, A.data_ptr(), k, Q.data_ptr(), k,
                                 R.data_ptr(), k, S.data_ptr(), k, ctypes.byref(o), st)
    L.check(rc, "tho_two_stage_noalloc")
    torch.cuda.synchronize()
    return to_host(Q), to_host(R), to_host(S)


def _same(a, b):
    for x, y in zip(a, b):
        assert x.shape == y.shape
        assert np.all(np.isfinite(x))
        assert np.array_equal(x, y), float(np.max(np.abs(x - y)))


def test_noalloc_matches_workspace_entry_point_two_calls():
    require_gpu()
    from paper_2602_14449_amd import _lib as L
    # the larger problem first (several chunks and tiles per chunk), then a
    # smaller one with other widths on the scratch the first call left behind
    for (n, k0, k, seed) in [(1 << 20, 64, 32, 71), (20000, 16, 8, 72)]:
        print("noalloc case n=%d k0=%d k=%d seed=%d" % (n, k0, k, seed), flush=True)
        g = np.random.default_rng(seed)
        V = to_dev(W.orthonormal(g, n, k0))
        A = to_dev(g.standard_normal((n, k)))
        ref = _with_workspace(L, L.THO_F64, V, A, n, k0, k)
        got = _noalloc(L, L.THO_F64, V, A, n, k0, k)
        _same(got, ref)


def test_noalloc_complex_and_limit():
    require_gpu()
    from paper_2602_14449_amd import _lib as L
    n, k0, k = 50000, 32, 16
    print("noalloc complex n=%d k0=%d k=%d" % (n, k0, k), flush=True)
    g = np.random.default_rng(73)
    V = to_dev(W.orthonormal(g, n, k0, complex_=True))
    A = to_dev((g.standard_normal((n, k)) + 1j * g.standard_normal((n, k))) / np.sqrt(2))
    _same(_noalloc(L, L.THO_C128, V, A, n, k0, k), _with_workspace(L, L.THO_C128, V, A, n, k0, k))
    # sizes whose workspace exceeds the fixed scratch are rejected before any work
    big = 1 << 22
    o = L.Opts()
    dummy = torch.empty(1, dtype=torch.float64, device="cuda")
    p = dummy.data_ptr()
    rc = L.tho_two_stage_noalloc(L.THO_F64, big, 128, 64, p, 128, p, 64, p, 64, p, 64, p, 64,
                                 ctypes.byref(o), torch.cuda.current_stream().cuda_stream)
    assert rc == -100
    assert b"fixed maximum" in L.tho_last_error()
