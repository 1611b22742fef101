"""Pins for the oracle's B-inner-product two-stage method (Algorithm 3, §5).

  * Theorem 4 on a densely formed H: H X = Y, H^* B H = B, and the inverse
    I - W T^{-*} W^* B;
  * B = I reduces Algorithm 3 to Algorithm 1 (the Euclidean oracle);
  * Algorithm 3 equals the plain definition computed through the Cholesky
    transform of the whole problem, for a dense SPD B with cond 1e5 (the B
    of Example 6), real and complex;
  * the B form of eq. (4) and [V, Q]^* B [V, Q] = I;
  * a diagonal B is the Euclidean method on rows scaled by sqrt(b) (the
    weighted inner product the GPU path implements).
"""

import numpy as np
import pytest

import tho_workloads as W
from oracle import two_stage
from oracle.b_inner import b_generalized_householder, b_qr, b_two_stage, b_two_stage_by_definition


def _spd(g, n, cond, cplx=False):
    X = W.orthonormal(g, n, n, complex_=cplx)
    d = 10.0 ** (-np.log10(cond) * np.arange(n) / (n - 1))
    B = (X * d[None, :]) @ np.conj(X).T
    return 0.5 * (B + np.conj(B).T)


def _case(n=300, k0=12, k=7, cond=1e5, cplx=False, seed=0):
    g = np.random.default_rng(seed)
    B = _spd(g, n, cond, cplx)
    V, _ = b_qr(B, W.gaussian(g, (n, k0), complex_=cplx))
    A = W.gaussian(g, (n, k), complex_=cplx)
    return B, V, A


def test_theorem4_dense_h():
    B, V, A = _case(n=40, k0=5, k=3)
    g = np.random.default_rng(1)
    # X with X^* B X = Y^* B Y = I
    X, _ = b_qr(B, g.standard_normal((40, 5)))
    H = b_generalized_householder(B, X, V)
    Wm = X - V
    T = Wm.T @ B @ X
    assert np.linalg.norm(H @ X - V) < 1e-12
    assert np.linalg.norm(H.T @ B @ H - B) < 1e-12 * np.linalg.norm(B)
    Hinv = np.eye(40) - Wm @ np.linalg.solve(T.T, Wm.T @ B)
    assert np.linalg.norm(Hinv @ H - np.eye(40)) < 1e-11


def test_identity_b_is_algorithm_1():
    g = np.random.default_rng(2)
    n, k0, k = 500, 10, 6
    V = W.orthonormal(g, n, k0)
    A = g.standard_normal((n, k))
    Qb, Rb, Sb = b_two_stage(np.eye(n), V, A)
    Q, R, S = two_stage(V, A)
    assert np.max(np.abs(Qb - Q)) < 1e-13 and np.max(np.abs(Rb - R)) < 1e-13 and np.max(np.abs(Sb - S)) < 1e-13


@pytest.mark.parametrize("cplx", [False, True])
def test_matches_definition_and_invariants(cplx):
    B, V, A = _case(cplx=cplx, seed=3)
    Q, R, S = b_two_stage(B, V, A)
    Qd, Rd, Sd = b_two_stage_by_definition(B, V, A)
    assert np.max(np.abs(Q - Qd)) < 1e-9 * np.max(np.abs(Qd))
    assert np.max(np.abs(R - Rd)) < 1e-10 * np.max(np.abs(Rd))
    assert np.max(np.abs(S - Sd)) < 1e-10 * np.max(np.abs(Sd))
    VQ = np.concatenate([V, Q], 1)
    G = np.conj(VQ).T @ B @ VQ
    assert np.linalg.norm(G - np.eye(G.shape[0]), 2) < 1e-12
    assert np.linalg.norm(A - V @ S - Q @ R) < 1e-12 * np.linalg.norm(A)
    assert np.allclose(np.tril(R, -1), 0) and np.all(np.real(np.diag(R)) >= 0)


def test_diagonal_b_is_scaled_euclidean():
    g = np.random.default_rng(4)
    n, k0, k = 800, 16, 8
    b = 10.0 ** g.uniform(-2, 2, n)
    V, _ = b_qr(np.diag(b), g.standard_normal((n, k0)))
    A = g.standard_normal((n, k))
    Q, R, S = b_two_stage(np.diag(b), V, A)
    s = np.sqrt(b)[:, None]
    Qt, Rt, St = two_stage(s * V, s * A)
    assert np.max(np.abs(Q - Qt / s)) < 1e-11 * np.max(np.abs(Q))
    assert np.max(np.abs(R - Rt)) < 1e-11 * np.max(np.abs(R))
    assert np.max(np.abs(S - St)) < 1e-11 * np.max(np.abs(S))
