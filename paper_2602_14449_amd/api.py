"""Argument marshalling between torch tensors and the libtho C ABI."""

import ctypes

import torch

from . import _lib as L


def _opts(panel="fp64"):
    o = L.Opts()
    o.p_choice = 0
    o.panel = L.PANELS[panel]
    o.flags = 0
    return o


def _dtype_code(t):
    if t.dtype == torch.float64:
        return L.THO_F64
    if t.dtype == torch.complex128:
        return L.THO_C128
    raise TypeError("tensors must be float64 or complex128, got %s" % t.dtype)


def _rowmajor(t, name):
    if t.dim() != 2:
        raise ValueError("%s must be 2-D" % name)
    if t.stride(1) != 1 and t.shape[1] > 1:
        raise ValueError("%s must have unit column stride" % name)
    return max(t.stride(0), t.shape[1], 1)


def workspace_bytes(n, k0, k, dtype=torch.float64, panel="fp64"):
    code = L.THO_F64 if dtype == torch.float64 else L.THO_C128
    nb = L.c_sz(0)
    o = _opts(panel)
    L.check(L.tho_two_stage_workspace(code, n, k0, k, ctypes.byref(o), ctypes.byref(nb)),
            "tho_two_stage_workspace")
    return nb.value


def two_stage(V, A, *, panel="fp64", out=None, workspace=None):
    """Algorithm 1 (second choice of P): returns (Q, R, S) with
    [V, A] = [V, Q] [[I, S], [0, R]] and [V, Q] orthonormal."""
    if not (V.is_cuda and A.is_cuda):
        raise ValueError("V and A must be GPU tensors")
    if V.dtype != A.dtype:
        raise TypeError("V and A must have the same dtype")
    code = _dtype_code(A)
    n, k0 = V.shape
    n2, k = A.shape
    if n2 != n:
        raise ValueError("V and A must have the same number of rows")
    ldv = _rowmajor(V, "V")
    lda = _rowmajor(A, "A")
    dev = A.device
    if out is None:
        Q = torch.empty((n, k), dtype=A.dtype, device=dev)
        R = torch.empty((k, k), dtype=A.dtype, device=dev)
        S = torch.empty((k0, k), dtype=A.dtype, device=dev)
    else:
        Q, R, S = out
    o = _opts(panel)
    nb = L.c_sz(0)
    L.check(L.tho_two_stage_workspace(code, n, k0, k, ctypes.byref(o), ctypes.byref(nb)),
            "tho_two_stage_workspace")
    if workspace is None or workspace.numel() < nb.value:
        workspace = torch.empty(max(nb.value, 1), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream(dev).cuda_stream
    rc = L.tho_two_stage(code, n, k0, k,
                         V.data_ptr() if k0 > 0 else None, ldv,
                         A.data_ptr(), lda,
                         Q.data_ptr(), max(k, 1),
                         R.data_ptr(), max(k, 1),
                         S.data_ptr() if k0 > 0 else None, max(k, 1),
                         ctypes.byref(o), workspace.data_ptr(), workspace.numel(),
                         stream)
    L.check(rc, "tho_two_stage")
    return Q, R, S
