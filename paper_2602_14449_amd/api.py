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


def _ld(t, name):
    """Row stride of a row-major 2-D tensor with unit column stride."""
    if t.dim() != 2:
        raise ValueError("%s must be 2-D" % name)
    if t.stride(1) != 1 and t.shape[1] > 1:
        raise ValueError("%s must have unit column stride" % name)
    return max(t.stride(0), t.shape[1], 1)


def _ptr(t, nonempty=True):
    return t.data_ptr() if (t is not None and (t.numel() > 0 or not nonempty)) else None


def _stream(dev):
    return torch.cuda.current_stream(dev).cuda_stream


def _check_inputs(V, A):
    if not (V.is_cuda and A.is_cuda):
        raise ValueError("V and A must be GPU tensors")
    if V.dtype != A.dtype:
        raise TypeError("V and A must have the same dtype")
    if V.shape[0] != A.shape[0]:
        raise ValueError("V and A must have the same number of rows")
    return _dtype_code(A), V.shape[0], V.shape[1], A.shape[1]


def _outputs(out, n, k0, k, like):
    if out is not None:
        return out
    return (torch.empty((n, k), dtype=like.dtype, device=like.device),
            torch.empty((k, k), dtype=like.dtype, device=like.device),
            torch.empty((k0, k), dtype=like.dtype, device=like.device))


def _workspace(nbytes, workspace, dev):
    if workspace is None or workspace.numel() < nbytes:
        workspace = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=dev)
    return workspace


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
    code, n, k0, k = _check_inputs(V, A)
    Q, R, S = _outputs(out, n, k0, k, A)
    o = _opts(panel)
    nb = L.c_sz(0)
    L.check(L.tho_two_stage_workspace(code, n, k0, k, ctypes.byref(o), ctypes.byref(nb)),
            "tho_two_stage_workspace")
    workspace = _workspace(nb.value, workspace, A.device)
    rc = L.tho_two_stage(code, n, k0, k,
                         _ptr(V), _ld(V, "V"), A.data_ptr(), _ld(A, "A"),
                         Q.data_ptr(), _ld(Q, "Q"), R.data_ptr(), _ld(R, "R"),
                         _ptr(S), _ld(S, "S") if k0 > 0 else max(k, 1),
                         ctypes.byref(o), workspace.data_ptr(), workspace.numel(),
                         _stream(A.device))
    L.check(rc, "tho_two_stage")
    return Q, R, S


def hhqr_full(V, A, *, out=None, workspace=None):
    """Householder QR of [V, A] (block Householder over 64-column panels):
    returns (Q, R, S) = (Q_B[:, k0:], R_B[k0:, k0:], R_B[:k0, k0:])."""
    code, n, k0, k = _check_inputs(V, A)
    Q, R, S = _outputs(out, n, k0, k, A)
    o = _opts()
    nb = L.c_sz(0)
    L.check(L.tho_hhqr_full_workspace(code, n, k0, k, ctypes.byref(o), ctypes.byref(nb)),
            "tho_hhqr_full_workspace")
    workspace = _workspace(nb.value, workspace, A.device)
    rc = L.tho_hhqr_full(code, n, k0, k,
                         _ptr(V), _ld(V, "V"), A.data_ptr(), _ld(A, "A"),
                         Q.data_ptr(), _ld(Q, "Q"), R.data_ptr(), _ld(R, "R"),
                         _ptr(S), _ld(S, "S") if k0 > 0 else max(k, 1),
                         ctypes.byref(o), workspace.data_ptr(), workspace.numel(),
                         _stream(A.device))
    L.check(rc, "tho_hhqr_full")
    return Q, R, S


def hhqr_full_workspace_bytes(n, k0, k):
    nb = L.c_sz(0)
    o = _opts()
    L.check(L.tho_hhqr_full_workspace(L.THO_F64, n, k0, k, ctypes.byref(o), ctypes.byref(nb)),
            "tho_hhqr_full_workspace")
    return nb.value


def bcgs(V, A, proj=1, rounds=1, *, out=None, workspace=None):
    """Block classical Gram-Schmidt baseline (eq. (1), Table 1 patterns):
    returns (Q, R, S) with A ~ V S + Q R."""
    code, n, k0, k = _check_inputs(V, A)
    Q, R, S = _outputs(out, n, k0, k, A)
    o = _opts()
    nb = L.c_sz(0)
    L.check(L.tho_bcgs_workspace(code, n, k0, k, proj, rounds, ctypes.byref(o), ctypes.byref(nb)),
            "tho_bcgs_workspace")
    workspace = _workspace(nb.value, workspace, A.device)
    rc = L.tho_bcgs(code, n, k0, k,
                    _ptr(V), _ld(V, "V"), A.data_ptr(), _ld(A, "A"),
                    Q.data_ptr(), _ld(Q, "Q"), R.data_ptr(), _ld(R, "R"),
                    _ptr(S), _ld(S, "S") if k0 > 0 else max(k, 1), proj, rounds,
                    ctypes.byref(o), workspace.data_ptr(), workspace.numel(),
                    _stream(A.device))
    L.check(rc, "tho_bcgs")
    return Q, R, S


def two_stage_backward(V, A, Q, R, gQ, gR, gS=None, *, workspace=None):
    """Adjoint of (V, A) -> (Q, R, S): returns (dV, dA) for the loss
    gradients gQ = dl/dQ, gR = dl/dR (upper triangle used), gS = dl/dS."""
    code, n, k0, k = _check_inputs(V, A)
    dV = torch.empty((n, k0), dtype=A.dtype, device=A.device)
    dA = torch.empty((n, k), dtype=A.dtype, device=A.device)
    o = _opts()
    nb = L.c_sz(0)
    L.check(L.tho_two_stage_backward_workspace(code, n, k0, k, ctypes.byref(o), ctypes.byref(nb)),
            "tho_two_stage_backward_workspace")
    workspace = _workspace(nb.value, workspace, A.device)
    gQ = gQ.contiguous()
    gR = gR.contiguous()
    if gS is not None:
        gS = gS.contiguous()
    rc = L.tho_two_stage_backward(
        code, n, k0, k,
        _ptr(V), _ld(V, "V"), A.data_ptr(), _ld(A, "A"),
        Q.data_ptr(), _ld(Q, "Q"), R.data_ptr(), _ld(R, "R"),
        gQ.data_ptr(), _ld(gQ, "gQ"), gR.data_ptr(), _ld(gR, "gR"),
        _ptr(gS) if (gS is not None and k0 > 0) else None,
        _ld(gS, "gS") if (gS is not None and k0 > 0) else max(k, 1),
        _ptr(dV), _ld(dV, "dV") if k0 > 0 else 1, dA.data_ptr(), _ld(dA, "dA"),
        ctypes.byref(o), workspace.data_ptr(), workspace.numel(), _stream(A.device))
    L.check(rc, "tho_two_stage_backward")
    return dV, dA


class TwoStageFunction(torch.autograd.Function):
    """(V, A) -> (Q, R, S) with the hand-written adjoint as its backward.
    Saves only V, A, Q, R; the WY factors are recomputed in the adjoint."""

    @staticmethod
    def forward(ctx, V, A):
        Q, R, S = two_stage(V.detach().contiguous(), A.detach().contiguous())
        ctx.save_for_backward(V, A, Q, R)
        return Q, R, S

    @staticmethod
    def backward(ctx, gQ, gR, gS):
        V, A, Q, R = ctx.saved_tensors
        if gQ is None:
            gQ = torch.zeros_like(Q)
        if gR is None:
            gR = torch.zeros_like(R)
        dV, dA = two_stage_backward(V.detach().contiguous(), A.detach().contiguous(), Q, R,
                                    gQ, gR, gS)
        return dV, dA


def two_stage_autograd(V, A):
    """Differentiable two_stage (real float64)."""
    if V.dtype != torch.float64 or A.dtype != torch.float64:
        raise TypeError("the adjoint is implemented for float64 only")
    return TwoStageFunction.apply(V, A)
