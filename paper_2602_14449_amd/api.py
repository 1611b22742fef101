"""Argument marshalling between torch tensors and the libtho C ABI."""

import ctypes

import torch

from . import _lib as L


def _opts(panel="fp64", p_choice="qr", check_finite=False, check_vorth=False):
    o = L.Opts()
    if p_choice not in L.PCHOICES:
        raise ValueError("p_choice must be one of %s" % sorted(L.PCHOICES))
    if panel not in L.PANELS:
        raise ValueError("panel must be one of %s" % sorted(L.PANELS))
    o.p_choice = L.PCHOICES[p_choice]
    o.panel = L.PANELS[panel]
    o.flags = (L.CHECK_FINITE if check_finite else 0) | (L.CHECK_VORTH if check_vorth else 0)
    return o


def _dtype_code(t):
    if t.dtype == torch.float64:
        return L.THO_F64
    if t.dtype == torch.complex128:
        return L.THO_C128
    raise TypeError("tensors must be float64 or complex128, got %s" % t.dtype)


def _ld(t, name):
    """Row stride of a row-major 2-D tensor with unit column stride.

    Rows must not overlap: a tensor with more than one row needs
    stride(0) >= shape[1] (an expanded or otherwise self-overlapping view
    would make the kernels read or write past its storage)."""
    if t.dim() != 2:
        raise ValueError("%s must be 2-D" % name)
    if t.stride(1) != 1 and t.shape[1] > 1:
        raise ValueError("%s must have unit column stride" % name)
    if t.shape[0] > 1 and t.shape[1] > 0 and t.stride(0) < t.shape[1]:
        raise ValueError("%s has overlapping rows (row stride %d < %d columns); pass a contiguous tensor"
                         % (name, t.stride(0), t.shape[1]))
    return max(t.stride(0), t.shape[1], 1)


def _check_out(t, shape, like, name):
    """An output tensor supplied by the caller must match exactly."""
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a tensor" % name)
    if tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))
    if t.dtype != like.dtype:
        raise TypeError("%s must have dtype %s, got %s" % (name, like.dtype, t.dtype))
    if t.device != like.device:
        raise ValueError("%s must be on %s, got %s" % (name, like.device, t.device))
    _ld(t, name)
    return t


def _ptr(t, nonempty=True):
    return t.data_ptr() if (t is not None and (t.numel() > 0 or not nonempty)) else None


def _stream(dev):
    return torch.cuda.current_stream(dev).cuda_stream


def _check_inputs(V, A):
    if not (isinstance(V, torch.Tensor) and isinstance(A, torch.Tensor)):
        raise TypeError("V and A must be tensors")
    if V.dim() != 2 or A.dim() != 2:
        raise ValueError("V and A must be 2-D")
    if V.dtype != A.dtype:
        raise TypeError("V and A must have the same dtype")
    if V.shape[0] != A.shape[0]:
        raise ValueError("V and A must have the same number of rows")
    code = _dtype_code(A)
    _ld(V, "V")
    _ld(A, "A")
    if not (V.is_cuda and A.is_cuda):
        raise ValueError("V and A must be GPU tensors")
    if V.device != A.device:
        raise ValueError("V and A must be on the same GPU")
    return code, V.shape[0], V.shape[1], A.shape[1]


def _outputs(out, n, k0, k, like):
    if out is not None:
        if len(out) != 3:
            raise ValueError("out must be a tuple (Q, R, S)")
        Q, R, S = out
        return (_check_out(Q, (n, k), like, "out Q"), _check_out(R, (k, k), like, "out R"),
                _check_out(S, (k0, k), like, "out S"))
    return (torch.empty((n, k), dtype=like.dtype, device=like.device),
            torch.empty((k, k), dtype=like.dtype, device=like.device),
            torch.empty((k0, k), dtype=like.dtype, device=like.device))


def _workspace(nbytes, workspace, dev):
    """A caller workspace is used when it is a byte tensor on `dev` that is
    large enough and contiguous; otherwise a new one is allocated."""
    if workspace is not None:
        if workspace.dtype != torch.uint8 or workspace.device != dev or not workspace.is_contiguous():
            raise ValueError("workspace must be a contiguous uint8 tensor on %s" % dev)
        if workspace.numel() >= nbytes:
            return workspace
    return torch.empty(max(nbytes, 1), dtype=torch.uint8, device=dev)


def workspace_bytes(n, k0, k, dtype=torch.float64, panel="fp64", p_choice="qr",
                    check_finite=False, check_vorth=False):
    code = L.THO_F64 if dtype == torch.float64 else L.THO_C128
    nb = L.c_sz(0)
    o = _opts(panel, p_choice, check_finite, check_vorth)
    L.check(L.tho_two_stage_workspace(code, n, k0, k, ctypes.byref(o), ctypes.byref(nb)),
            "tho_two_stage_workspace")
    return nb.value


def two_stage(V, A, *, p_choice="qr", panel="fp64", check_finite=False, check_vorth=False,
              out=None, workspace=None):
    """Algorithm 1: returns (Q, R, S) with [V, A] = [V, Q] [[I, S], [0, R]]
    and [V, Q] orthonormal.  p_choice: "qr" (second choice of P, default),
    "mlu" (first choice, modified LU) or "polar" (third choice).
    check_finite / check_vorth ask the library to record a non-finite input
    or a V with ||V^T V - I||_F above 1e-10 in the workspace's info word; pass
    your own ``workspace`` and read it with ``get_info(workspace)``."""
    code, n, k0, k = _check_inputs(V, A)
    Q, R, S = _outputs(out, n, k0, k, A)
    o = _opts(panel, p_choice, check_finite, check_vorth)
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


def block_householder(A, block_sizes, *, p_choice="qr", out=None, workspace=None):
    """Algorithm 4 (block Householder-QR) of the column blocks of A (widths
    ``block_sizes``, each <= 64): returns (Q, R) with A = Q R, Q^T Q = I, R
    upper triangular with nonnegative diagonal."""
    if not isinstance(A, torch.Tensor) or A.dim() != 2 or not A.is_cuda:
        raise ValueError("A must be a 2-D GPU tensor")
    if A.dtype != torch.float64:
        raise TypeError("block_householder supports float64 only")
    n, kt = A.shape
    kb = [int(b) for b in block_sizes]
    if sum(kb) != kt:
        raise ValueError("block sizes must add up to the number of columns")
    if out is not None:
        Q, R = out
        _check_out(Q, (n, kt), A, "out Q")
        _check_out(R, (kt, kt), A, "out R")
    else:
        Q = torch.empty((n, kt), dtype=A.dtype, device=A.device)
        R = torch.empty((kt, kt), dtype=A.dtype, device=A.device)
    o = _opts("fp64", p_choice)
    nb = L.c_sz(0)
    L.check(L.tho_block_householder_workspace(L.THO_F64, n, kt, ctypes.byref(o), ctypes.byref(nb)),
            "tho_block_householder_workspace")
    workspace = _workspace(nb.value, workspace, A.device)
    arr = (L.c_i64 * max(len(kb), 1))(*kb)
    rc = L.tho_block_householder(L.THO_F64, n, len(kb), arr, A.data_ptr(), _ld(A, "A"), Q.data_ptr(), _ld(Q, "Q"),
                                 R.data_ptr(), _ld(R, "R"), ctypes.byref(o), workspace.data_ptr(),
                                 workspace.numel(), _stream(A.device))
    L.check(rc, "tho_block_householder")
    return Q, R


class BlockHouseholder:
    """Incremental Algorithm 4: ``append(A_i)`` orthogonalizes one more block
    against the basis built so far and returns (Q_i, R_col_i), the new basis
    columns and the rows 0 .. c_i + k_i - 1 of R's block column."""

    def __init__(self, n, kmax, *, device="cuda", p_choice="qr"):
        self.n, self.kmax = int(n), int(kmax)
        dev = torch.device(device)
        if dev.type == "cuda" and dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        self.opts = _opts("fp64", p_choice)
        nb = L.c_sz(0)
        L.check(L.tho_block_householder_workspace(L.THO_F64, self.n, self.kmax, ctypes.byref(self.opts),
                                                  ctypes.byref(nb)), "tho_block_householder_workspace")
        self.ws = torch.empty(max(nb.value, 1), dtype=torch.uint8, device=self.device)
        self.Q = torch.zeros((self.n, self.kmax), dtype=torch.float64, device=self.device)
        self.R = torch.zeros((self.kmax, self.kmax), dtype=torch.float64, device=self.device)
        self.widths = []

    @property
    def ncols(self):
        return sum(self.widths)

    def append(self, Ai):
        if Ai.dtype != torch.float64 or Ai.device != self.device or Ai.dim() != 2 or Ai.shape[0] != self.n:
            raise ValueError("A_i must be a float64 (n, k_i) tensor on %s" % self.device)
        c0, ki = self.ncols, Ai.shape[1]
        if c0 + ki > self.kmax:
            raise ValueError("basis would exceed kmax = %d columns" % self.kmax)
        kb = self.widths + [ki]
        arr = (L.c_i64 * len(kb))(*kb)
        rc = L.tho_block_householder_step(L.THO_F64, self.n, len(kb) - 1, arr, self.kmax, Ai.data_ptr(),
                                          _ld(Ai, "A_i"), self.Q.data_ptr(), self.kmax, self.R.data_ptr(),
                                          self.kmax, ctypes.byref(self.opts), self.ws.data_ptr(), self.ws.numel(),
                                          _stream(self.device))
        L.check(rc, "tho_block_householder_step")
        self.widths.append(ki)
        return self.Q[:, c0:c0 + ki], self.R[:c0 + ki, c0:c0 + ki]


def two_stage_weighted(V, A, b, *, p_choice="qr", check_finite=False, check_vorth=False, out=None,
                       workspace=None):
    """Two-stage method in the weighted inner product <x, y> = x^* diag(b) y
    (Algorithm 3 with a diagonal B): returns (Q, R, S) with
    [V, A] = [V, Q] [[I, S], [0, R]] and [V, Q]^* diag(b) [V, Q] = I."""
    code, n, k0, k = _check_inputs(V, A)
    if not isinstance(b, torch.Tensor) or b.dtype != torch.float64 or b.shape != (n,) or b.device != A.device:
        raise ValueError("b must be a float64 tensor of shape (n,) on the inputs' device")
    b = b.contiguous()
    Q, R, S = _outputs(out, n, k0, k, A)
    o = _opts("fp64", p_choice, check_finite, check_vorth)
    nb = L.c_sz(0)
    L.check(L.tho_two_stage_weighted_workspace(code, n, k0, k, ctypes.byref(o), ctypes.byref(nb)),
            "tho_two_stage_weighted_workspace")
    workspace = _workspace(nb.value, workspace, A.device)
    rc = L.tho_two_stage_weighted(code, n, k0, k, b.data_ptr(),
                                  _ptr(V), _ld(V, "V"), A.data_ptr(), _ld(A, "A"),
                                  Q.data_ptr(), _ld(Q, "Q"), R.data_ptr(), _ld(R, "R"),
                                  _ptr(S), _ld(S, "S") if k0 > 0 else max(k, 1),
                                  ctypes.byref(o), workspace.data_ptr(), workspace.numel(), _stream(A.device))
    L.check(rc, "tho_two_stage_weighted")
    return Q, R, S


def get_info(workspace=None):
    """Info word of the last two_stage call on ``workspace`` (None: the
    static scratch of the no-allocation entry point on the current device):
    0, INFO_NONFINITE (1) or INFO_V_NOT_ORTHONORMAL (3).  Synchronizes the
    current stream first."""
    torch.cuda.current_stream().synchronize()
    v = L.c_i32(0)
    L.check(L.tho_get_info(workspace.data_ptr() if workspace is not None else None, ctypes.byref(v)),
            "tho_get_info")
    return v.value


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
    gradients gQ = dl/dQ, gR = dl/dR (upper triangle used), gS = dl/dS.
    Complex data: dl = Re<dV, dV_dir> + Re<dA, dA_dir> with <X, Y> =
    sum conj(X) Y, for l = Re<gQ, Q> + Re<gR, R> + Re<gS, S>."""
    code, n, k0, k = _check_inputs(V, A)
    _check_out(Q, (n, k), A, "Q")
    _check_out(R, (k, k), A, "R")
    _check_out(gQ, (n, k), A, "gQ")
    _check_out(gR, (k, k), A, "gR")
    if gS is not None:
        _check_out(gS, (k0, k), A, "gS")
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


class BatchedPlan:
    """Many independent two-stage problems (V_i, A_i) in one persistent,
    graph-captured launch.  Allocates the outputs and the workspace, binds
    them into a plan (autotuned at creation) and replays it with run()."""

    def __init__(self, pairs):
        if len(pairs) == 0:
            raise ValueError("empty batch")
        dev = pairs[0][1].device
        self.pairs = pairs
        self.outputs = []
        probs = (L.Problem * len(pairs))()
        for i, (V, A) in enumerate(pairs):
            if V.dtype != torch.float64 or A.dtype != torch.float64:
                raise TypeError("the batched path is real float64")
            if not (V.is_cuda and A.is_cuda and A.device == dev and V.device == dev):
                raise ValueError("all tensors must be on the same GPU")
            n, k0 = V.shape
            k = A.shape[1]
            Q = torch.empty((n, k), dtype=A.dtype, device=dev)
            R = torch.empty((k, k), dtype=A.dtype, device=dev)
            S = torch.empty((k0, k), dtype=A.dtype, device=dev)
            self.outputs.append((Q, R, S))
            p = probs[i]
            p.n, p.k0, p.k = n, k0, k
            p.V, p.ldv = _ptr(V), _ld(V, "V")
            p.A, p.lda = _ptr(A), _ld(A, "A")
            p.Q, p.ldq = _ptr(Q), _ld(Q, "Q")
            p.R, p.ldr = _ptr(R), _ld(R, "R")
            p.S, p.lds = _ptr(S), (_ld(S, "S") if k0 > 0 else max(k, 1))
        self._probs = probs
        o = _opts()
        nb = L.c_sz(0)
        L.check(L.tho_batched_workspace(len(pairs), probs, ctypes.byref(o), ctypes.byref(nb)),
                "tho_batched_workspace")
        self.workspace = torch.empty(max(nb.value, 1), dtype=torch.uint8, device=dev)
        self.device = dev
        h = L.c_vp()
        L.check(L.tho_batched_plan_create(len(pairs), probs, self.workspace.data_ptr(),
                                          self.workspace.numel(), ctypes.byref(o), _stream(dev),
                                          ctypes.byref(h)), "tho_batched_plan_create")
        self._plan = h

    def run(self):
        L.check(L.tho_batched_run(self._plan, _stream(self.device)), "tho_batched_run")
        return self.outputs

    def info(self):
        tr, gr, ms = L.c_i32(0), L.c_i32(0), ctypes.c_double(0)
        L.check(L.tho_batched_plan_info(self._plan, ctypes.byref(tr), ctypes.byref(gr), ctypes.byref(ms)),
                "tho_batched_plan_info")
        return {"tile_rows": tr.value, "workgroups": gr.value, "tuned_ms": ms.value}

    def close(self):
        if getattr(self, "_plan", None):
            torch.cuda.synchronize(self.device)
            L.tho_plan_destroy(self._plan)
            self._plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def two_stage_batched(pairs):
    """Two-stage orthogonalization of every (V_i, A_i): list of (Q, R, S)."""
    plan = BatchedPlan(pairs)
    out = plan.run()
    plan.close()
    return out


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
    """Differentiable two_stage (float64 or complex128; for complex data the
    gradients follow PyTorch's convention for real losses)."""
    if V.dtype != A.dtype or A.dtype not in (torch.float64, torch.complex128):
        raise TypeError("the adjoint is implemented for float64 and complex128")
    return TwoStageFunction.apply(V, A)
