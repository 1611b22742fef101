"""GPU parity of the complex128 adjoint (tho_two_stage_backward with
THO_C128) and of the autograd Function on complex tensors.

Element-wise against the oracle's complex reverse-mode gradient (pinned on
the CPU by complex central differences and PyTorch autograd), and against
central finite differences of the GPU forward pass itself along complex
directions (step 1e-6, n = 256, k0 = 8, k = 4).  Convention: for
l = Re<G_Q, Q> + Re<G_R, R> + Re<G_S, S>, dl = Re<dV, dV_dir> + Re<dA, dA_dir>.
"""

import numpy as np
import pytest
import torch

import tho_workloads as W
from oracle.adjoint import two_stage_vjp

from gpu_util import require_gpu, to_dev, to_host

pytestmark = pytest.mark.gpu


def _zg(g, shape):
    return W.gaussian(g, shape, complex_=True)


def _grads(V, A, GQ, GR, GS):
    import paper_2602_14449_amd as tho
    Vd, Ad = to_dev(V), to_dev(A)
    Q, R, S = tho.two_stage(Vd, Ad)
    dV, dA = tho.two_stage_backward(Vd, Ad, Q, R, to_dev(GQ), to_dev(GR),
                                    None if GS is None else to_dev(GS))
    return to_host(dV), to_host(dA)


def _rel(x, ref):
    return np.abs(x - ref).max() / max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("n,k0,k,with_gs", [
    (256, 8, 4, False), (3000, 16, 8, True), (4100, 33, 17, False), (20000, 64, 32, True),
    (2000, 0, 16, False), (600, 64, 32, True), (70001, 48, 20, False)])
def test_complex_backward_parity(n, k0, k, with_gs):
    require_gpu()
    print("complex adjoint n=%d k0=%d k=%d gS=%s" % (n, k0, k, with_gs), flush=True)
    g = np.random.default_rng(900 + n + k0 + k)
    V = W.orthonormal(g, n, k0, complex_=True)
    A, GQ, GR = _zg(g, (n, k)), _zg(g, (n, k)), _zg(g, (k, k))
    GS = _zg(g, (k0, k)) if with_gs else None
    dV, dA = _grads(V, A, GQ, GR, GS)
    rV, rA = two_stage_vjp(V, A, GQ, GR, GS)
    eA = _rel(dA, rA)
    eV = _rel(dV, rV) if k0 else 0.0
    print("rel err dA %.2e dV %.2e" % (eA, eV))
    assert eA < 1e-9 and eV < 1e-9


def test_complex_backward_fd_of_gpu_forward():
    require_gpu()
    import paper_2602_14449_amd as tho
    g = np.random.default_rng(31)
    n, k0, k = 256, 8, 4
    V = W.orthonormal(g, n, k0, complex_=True)
    A, GQ, GR, GS = _zg(g, (n, k)), _zg(g, (n, k)), _zg(g, (k, k)), _zg(g, (k0, k))
    dV, dA = _grads(V, A, GQ, GR, GS)

    def loss(Vx, Ax):
        Q, R, S = tho.two_stage(to_dev(Vx), to_dev(Ax))
        Q, R, S = to_host(Q), to_host(R), to_host(S)
        return float(np.real(np.sum(np.conj(GQ) * Q) + np.sum(np.conj(GR) * np.triu(R)) + np.sum(np.conj(GS) * S)))
    h = 1e-6
    for _ in range(3):
        DV, DA = _zg(g, V.shape), _zg(g, A.shape)
        fd = (loss(V + h * DV, A + h * DA) - loss(V - h * DV, A - h * DA)) / (2 * h)
        an = float(np.real(np.sum(np.conj(dV) * DV) + np.sum(np.conj(dA) * DA)))
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (fd, an)


def test_complex_autograd_function():
    require_gpu()
    import paper_2602_14449_amd as tho
    g = np.random.default_rng(32)
    n, k0, k = 5000, 24, 12
    V = W.orthonormal(g, n, k0, complex_=True)
    A, GQ, GR = _zg(g, (n, k)), _zg(g, (n, k)), _zg(g, (k, k))
    Vd = to_dev(V).requires_grad_(True)
    Ad = to_dev(A).requires_grad_(True)
    Q, R, S = tho.two_stage_autograd(Vd, Ad)
    l = ((to_dev(GQ).conj() * Q).sum() + (to_dev(GR).conj() * torch.triu(R)).sum()).real
    l.backward()
    rV, rA = two_stage_vjp(V, A, GQ, GR)
    assert _rel(to_host(Vd.grad), rV) < 1e-9 and _rel(to_host(Ad.grad), rA) < 1e-9
