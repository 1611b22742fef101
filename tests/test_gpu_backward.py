"""GPU parity of the hand-written adjoint (tho_two_stage_backward) and of the
autograd Function built on it.

Element-wise against the oracle's reverse-mode gradient of Algorithm 1
(second choice of P), and against central finite differences of the GPU
forward pass itself (step 1e-6, n = 256, k0 = 8, k = 4).
"""

import numpy as np
import pytest
import torch

import tho_workloads as W
from oracle.adjoint import two_stage_vjp

from gpu_util import require_gpu, to_dev, to_host

pytestmark = pytest.mark.gpu


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
    (5000, 128, 64, False), (2000, 0, 16, False), (600, 128, 64, True), (70001, 64, 40, False)])
def test_backward_parity(n, k0, k, with_gs):
    require_gpu()
    g = np.random.default_rng(700 + n + k0 + k)
    V = W.orthonormal(g, n, k0)
    A = g.standard_normal((n, k))
    GQ = g.standard_normal((n, k))
    GR = g.standard_normal((k, k))
    GS = g.standard_normal((k0, k)) if with_gs else None
    dV, dA = _grads(V, A, GQ, GR, GS)
    rV, rA = two_stage_vjp(V, A, GQ, GR, GS)
    assert dA.shape == rA.shape and dV.shape == rV.shape
    eA = _rel(dA, rA)
    eV = _rel(dV, rV) if k0 else 0.0
    print("rel err dA %.2e dV %.2e" % (eA, eV))
    assert eA < 1e-9
    assert eV < 1e-9


def test_backward_full_size_grad_workload():
    # n = 2^20, k0 = 64, k = 32 with Gaussian G_Q, G_R (the differentiation
    # workload), element-wise against the oracle at full size
    require_gpu()
    V, A, GQ, GR = W.grad_case()
    dV, dA = _grads(V, A, GQ, GR, None)
    rV, rA = two_stage_vjp(V, A, GQ, GR, None)
    eA, eV = _rel(dA, rA), _rel(dV, rV)
    print("rel err dA %.2e dV %.2e" % (eA, eV))
    assert eA < 1e-9
    assert eV < 1e-9


def test_autograd_against_central_differences():
    require_gpu()
    import paper_2602_14449_amd as tho
    g = np.random.default_rng(31)
    n, k0, k = 256, 8, 4
    V = W.orthonormal(g, n, k0)
    A = g.standard_normal((n, k))
    GQ = to_dev(g.standard_normal((n, k)))
    GR = to_dev(np.triu(g.standard_normal((k, k))))
    Vd = to_dev(V).requires_grad_(True)
    Ad = to_dev(A).requires_grad_(True)
    Q, R, S = tho.two_stage_autograd(Vd, Ad)
    loss = (GQ * Q).sum() + (GR * R).sum()
    loss.backward()

    def f(Vx, Ax):
        with torch.no_grad():
            Qx, Rx, _ = tho.two_stage(Vx, Ax)
            return float((GQ * Qx).sum() + (GR * Rx).sum())

    h = 1e-6
    for trial in range(4):
        dVd = to_dev(g.standard_normal((n, k0)))
        dAd = to_dev(g.standard_normal((n, k)))
        fd = (f(to_dev(V) + h * dVd, to_dev(A) + h * dAd) -
              f(to_dev(V) - h * dVd, to_dev(A) - h * dAd)) / (2 * h)
        an = float((Vd.grad * dVd).sum() + (Ad.grad * dAd).sum())
        print("trial", trial, "fd", fd, "adjoint", an)
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))
