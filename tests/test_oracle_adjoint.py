"""Pins for the oracle's reverse-mode gradient of Algorithm 1 (CPU only).

The paper is silent on gradients; the reading is that the gradient is that of
the map the oracle's Algorithm 1 computes.  Pins:
  * brute force: central finite differences (step 1e-6) of the forward oracle
    at n=256, k0=8, k=4 along random directions and sampled coordinates;
  * a library routine: PyTorch CPU autograd through an independent torch
    transcription of Algorithm 1 (torch.linalg.qr with the sign fix);
  * the special case k0 = 0, which is plain QR: torch.linalg.qr's backward;
  * the QR adjoint alone against finite differences.
"""

import numpy as np
import pytest
import torch

import tho_workloads as W
from oracle.adjoint import two_stage_vjp, central_fd, qr_adjoint
from oracle.householder import qr_pos


def _case(n=256, k0=8, k=4, seed=0):
    g = np.random.default_rng(seed)
    V = W.orthonormal(g, n, k0)
    A = g.standard_normal((n, k))
    GQ = g.standard_normal((n, k))
    GR = g.standard_normal((k, k))
    GS = g.standard_normal((k0, k))
    return g, V, A, GQ, GR, GS


@pytest.mark.parametrize("with_gs", [False, True])
def test_fd_random_directions(with_gs):
    g, V, A, GQ, GR, GS = _case()
    GS = GS if with_gs else None
    Vb, Ab = two_stage_vjp(V, A, GQ, GR, GS)
    for _ in range(4):
        dV = g.standard_normal(V.shape)
        dA = g.standard_normal(A.shape)
        fd = central_fd(V, A, GQ, GR, GS, dV, dA, h=1e-6)
        an = np.sum(Vb * dV) + np.sum(Ab * dA)
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (fd, an)


def test_fd_sampled_coordinates():
    g, V, A, GQ, GR, GS = _case(seed=1)
    Vb, Ab = two_stage_vjp(V, A, GQ, GR, GS)
    coords = [(0, 0), (3, 7), (7, 2), (8, 1), (100, 5), (255, 7)]
    for (i, j) in coords:
        dV = np.zeros_like(V)
        dV[i, j] = 1.0
        fd = central_fd(V, A, GQ, GR, GS, dV, np.zeros_like(A), h=1e-6)
        assert abs(fd - Vb[i, j]) <= 1e-6 * max(1.0, abs(Vb[i, j]))
    for (i, j) in [(0, 0), (5, 3), (200, 1)]:
        dA = np.zeros_like(A)
        dA[i, j] = 1.0
        fd = central_fd(V, A, GQ, GR, GS, np.zeros_like(V), dA, h=1e-6)
        assert abs(fd - Ab[i, j]) <= 1e-6 * max(1.0, abs(Ab[i, j]))


def _torch_qr_pos(X):
    Q, R = torch.linalg.qr(X, mode="reduced")
    d = torch.sign(torch.diagonal(R))
    d = torch.where(d == 0, torch.ones_like(d), d)
    return Q * d[None, :], d[:, None] * R


def _torch_two_stage(V, A):
    # an independent transcription of Algorithm 1 (second choice of P)
    n, k0 = V.shape
    k = A.shape[1]
    Q1, R1 = _torch_qr_pos(V[:k0])
    P = -Q1
    X0 = torch.cat([P, torch.zeros(n - k0, k0, dtype=V.dtype)], 0)
    Wm = X0 - V
    T = torch.eye(k0, dtype=V.dtype) + R1.T
    Z = torch.linalg.solve_triangular(T.T, Wm.T @ A, upper=True)
    A1 = A - Wm @ Z
    S = P.T @ A1[:k0]
    Qu, R = _torch_qr_pos(A1[k0:])
    Xq = torch.cat([torch.zeros(k0, k, dtype=V.dtype), Qu], 0)
    N = torch.linalg.solve_triangular(T, Wm.T @ Xq, upper=False)
    Q = Xq - Wm @ N
    return Q, R, S


def test_matches_torch_autograd():
    _, V, A, GQ, GR, GS = _case(seed=2)
    Vt = torch.tensor(V, requires_grad=True)
    At = torch.tensor(A, requires_grad=True)
    Q, R, S = _torch_two_stage(Vt, At)
    loss = (torch.tensor(GQ) * Q).sum() + (torch.tensor(GR) * R).sum() \
        + (torch.tensor(GS) * S).sum()
    loss.backward()
    Vb, Ab = two_stage_vjp(V, A, GQ, GR, GS)
    assert np.allclose(Vb, Vt.grad.numpy(), rtol=1e-10, atol=1e-10)
    assert np.allclose(Ab, At.grad.numpy(), rtol=1e-10, atol=1e-10)


def test_k0_zero_equals_torch_qr_backward():
    g = np.random.default_rng(3)
    A = g.standard_normal((64, 6))
    GQ = g.standard_normal((64, 6))
    GR = g.standard_normal((6, 6))
    At = torch.tensor(A, requires_grad=True)
    Q, R = _torch_qr_pos(At)
    ((torch.tensor(GQ) * Q).sum() + (torch.tensor(GR) * R).sum()).backward()
    _, Ab = two_stage_vjp(np.zeros((64, 0)), A, GQ, GR)
    assert np.allclose(Ab, At.grad.numpy(), rtol=1e-11, atol=1e-11)


def test_qr_adjoint_fd():
    g = np.random.default_rng(4)
    X = g.standard_normal((30, 5))
    Qb = g.standard_normal((30, 5))
    Rb = g.standard_normal((5, 5))
    Q, R = qr_pos(X)
    Xb = qr_adjoint(Q, R, Qb, Rb)
    D = g.standard_normal(X.shape)
    h = 1e-6

    def f(Y):
        q, r = qr_pos(Y)
        return np.sum(q * Qb) + np.sum(np.triu(r) * Rb)
    fd = (f(X + h * D) - f(X - h * D)) / (2 * h)
    assert abs(fd - np.sum(Xb * D)) < 1e-7 * max(1, abs(fd))


# ------------------------------------------------------- complex128
# Gradient convention for complex data: dl = Re<V_bar, dV> + Re<A_bar, dA>
# with <X, Y> = sum conj(X) Y and l = Re<G_Q, Q> + Re<G_R, R> + Re<G_S, S>
# (PyTorch's convention for real losses of complex tensors).

def _zcase(n=256, k0=8, k=4, seed=10):
    g = np.random.default_rng(seed)
    V = W.orthonormal(g, n, k0, complex_=True)
    A = W.gaussian(g, (n, k), complex_=True)
    GQ = W.gaussian(g, (n, k), complex_=True)
    GR = W.gaussian(g, (k, k), complex_=True)
    GS = W.gaussian(g, (k0, k), complex_=True)
    return g, V, A, GQ, GR, GS


def _re_inner(X, Y):
    return float(np.real(np.sum(np.conj(X) * Y)))


@pytest.mark.parametrize("with_gs", [False, True])
def test_complex_fd_random_directions(with_gs):
    g, V, A, GQ, GR, GS = _zcase()
    GS = GS if with_gs else None
    Vb, Ab = two_stage_vjp(V, A, GQ, GR, GS)
    for _ in range(4):
        dV = W.gaussian(g, V.shape, complex_=True)
        dA = W.gaussian(g, A.shape, complex_=True)
        fd = central_fd(V, A, GQ, GR, GS, dV, dA, h=1e-6)
        an = _re_inner(Vb, dV) + _re_inner(Ab, dA)
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (fd, an)


def test_complex_fd_sampled_coordinates_real_and_imaginary():
    g, V, A, GQ, GR, GS = _zcase(seed=11)
    Vb, Ab = two_stage_vjp(V, A, GQ, GR, GS)
    for (i, j) in [(0, 0), (3, 7), (9, 2), (200, 5)]:
        for unit in (1.0, 1j):
            dV = np.zeros_like(V)
            dV[i, j] = unit
            fd = central_fd(V, A, GQ, GR, GS, dV, np.zeros_like(A), h=1e-6)
            assert abs(fd - _re_inner(Vb, dV)) <= 1e-6 * max(1.0, abs(Vb[i, j]))
    for (i, j) in [(1, 0), (100, 3)]:
        for unit in (1.0, 1j):
            dA = np.zeros_like(A)
            dA[i, j] = unit
            fd = central_fd(V, A, GQ, GR, GS, np.zeros_like(V), dA, h=1e-6)
            assert abs(fd - _re_inner(Ab, dA)) <= 1e-6 * max(1.0, abs(Ab[i, j]))


def _torch_zqr_pos(X):
    Q, R = torch.linalg.qr(X, mode="reduced")
    d = torch.diagonal(R)
    ph = torch.where(d.abs() > 0, d / d.abs(), torch.ones_like(d))
    return Q * ph[None, :], ph.conj()[:, None] * R


def _torch_ztwo_stage(V, A):
    # an independent transcription of the method for complex data
    n, k0 = V.shape
    k = A.shape[1]
    Q1, R1 = _torch_zqr_pos(V[:k0])
    P = -Q1
    Wm = torch.cat([P, torch.zeros(n - k0, k0, dtype=V.dtype)], 0) - V
    T = torch.eye(k0, dtype=V.dtype) + R1.mH
    Z = torch.linalg.solve_triangular(T.mH, Wm.mH @ A, upper=True)
    A1 = A - Wm @ Z
    S = P.mH @ A1[:k0]
    Qu, R = _torch_zqr_pos(A1[k0:])
    Xq = torch.cat([torch.zeros(k0, k, dtype=V.dtype), Qu], 0)
    N = torch.linalg.solve_triangular(T, Wm.mH @ Xq, upper=False)
    return Xq - Wm @ N, R, S


def test_complex_matches_torch_autograd():
    _, V, A, GQ, GR, GS = _zcase(n=128, k0=6, k=3, seed=12)
    Vt = torch.tensor(V, requires_grad=True)
    At = torch.tensor(A, requires_grad=True)
    Q, R, S = _torch_ztwo_stage(Vt, At)
    loss = ((torch.tensor(GQ).conj() * Q).sum() + (torch.tensor(GR).conj() * torch.triu(R)).sum()
            + (torch.tensor(GS).conj() * S).sum()).real
    loss.backward()
    Vb, Ab = two_stage_vjp(V, A, GQ, GR, GS)
    assert np.max(np.abs(Vb - Vt.grad.numpy())) < 1e-11 * np.max(np.abs(Vb))
    assert np.max(np.abs(Ab - At.grad.numpy())) < 1e-11 * np.max(np.abs(Ab))


def test_complex_k0_zero_equals_torch_qr_backward():
    g = np.random.default_rng(13)
    A = W.gaussian(g, (64, 6), complex_=True)
    GQ = W.gaussian(g, (64, 6), complex_=True)
    GR = W.gaussian(g, (6, 6), complex_=True)
    At = torch.tensor(A, requires_grad=True)
    Q, R = _torch_zqr_pos(At)
    ((torch.tensor(GQ).conj() * Q).sum() + (torch.tensor(GR).conj() * torch.triu(R)).sum()).real.backward()
    _, Ab = two_stage_vjp(np.zeros((64, 0), dtype=np.complex128), A, GQ, GR)
    assert np.max(np.abs(Ab - At.grad.numpy())) < 1e-11 * np.max(np.abs(Ab))
