"""Algorithm 1 (two-stage Householder-QR) with the second choice of P (oracle).

Test infrastructure only (see ``oracle/__init__``).

Followed passages
  * §3.1: generalized Householder transformation H = I - W T^{-1} W^* with
    X = [P; 0], Y = V, W = X - Y, T = W^* X (eq. (3)); stage two forms
    H^* A, QRs its bottom n - k0 rows and sets Q = H [0; Q_], giving eq. (4):
    [V, A] = [V, Q] [[I, S], [0, R]].
  * Algorithm 1, steps in order: choose unitary P; W = [P; 0] - V;
    T = I - V_top^* P; A <- (I - W T^{-*} W^*) A; S = P^* A_top;
    QR of A_low = Q_ R; Q = (I - W T^{-1} W^*) [0; Q_].
  * §3.2, second choice: V_top = Q1 R1 with nonnegative diag(R1), P = -Q1,
    T = I + R1^* (lower triangular).  Appendix B.2 analyses exactly the
    computed form T = fl(I + R1^*), which is the form used here.  (Algorithm 1 itself
    writes T = I - V_top^* P, equal whenever Q1 is unitary; the
    tests check the two agree to rounding.)

Readings taken where the paper is silent (listed in the design doc as well)
  * Intra-block QR: column Householder with the nonnegative-diagonal phase
    convention (``householder.qr_pos``).
  * S is computed exactly as Algorithm 1 states, P^* A_top after the update, not
    as V^* A (they agree in exact arithmetic when V^* V = I).
  * n >= k0 + k is required; k0 = 0 reduces to qr_pos(A); k = 0 is a no-op.
"""

import numpy as np
from scipy.linalg import solve_triangular

from .householder import qr_pos


def _h(M):
    return np.conj(M).T


def two_stage_intermediates(V, A, qr_method="auto"):
    """Run Algorithm 1 (second choice of P) and return every intermediate.

    Returns a dict with P, T, W, Y (= W^* A), Z (= T^{-*} Y), A1 (updated A),
    S, Qu (Q_ of the bottom-block QR), R, G (= W^* [0; Q_]), N (= T^{-1} G) and Q.
    """
    V = np.asarray(V)
    A = np.asarray(A)
    dt = np.result_type(V, A, np.float64)
    V = V.astype(dt, copy=False)
    A = A.astype(dt, copy=False)
    n, k0 = V.shape
    n2, k = A.shape
    if n2 != n:
        raise ValueError("V and A must have the same number of rows")
    if n < k0 + k:
        raise ValueError("need n >= k0 + k")
    out = {}
    # choice of P, second choice (§3.2): V_top = Q1 R1, diag(R1) >= 0, P = -Q1
    if k0 > 0:
        Q1, R1 = qr_pos(V[:k0, :], method="loop")
    else:
        Q1 = np.zeros((0, 0), dt)
        R1 = np.zeros((0, 0), dt)
    P = -Q1
    # W = [P; 0] - V
    X0 = np.zeros((n, k0), dt)
    X0[:k0, :] = P
    W = X0 - V
    # T in the form analysed in Appendix B.2: T = I + R1^* (lower tri.)
    T = np.eye(k0, dtype=dt) + _h(R1)
    # update of A: A <- A - W T^{-*} (W^* A)
    Y = _h(W) @ A
    if k0 > 0:
        Z = solve_triangular(_h(T), Y, lower=False)   # T^* is upper triangular
    else:
        Z = np.zeros((0, k), dt)
    A1 = A - W @ Z
    # S = P^* A_top
    S = _h(P) @ A1[:k0, :]
    # QR of the bottom n - k0 rows
    if k > 0:
        Qu, R = qr_pos(A1[k0:, :], method=qr_method)
    else:
        Qu = np.zeros((n - k0, 0), dt)
        R = np.zeros((0, 0), dt)
    # formation of Q: Q = [0; Q_] - W T^{-1} (W^* [0; Q_])
    Xq = np.zeros((n, k), dt)
    Xq[k0:, :] = Qu
    G = _h(W) @ Xq
    if k0 > 0:
        N = solve_triangular(T, G, lower=True)
    else:
        N = np.zeros((0, k), dt)
    Q = Xq - W @ N
    out.update(P=P, R1=R1, T=T, W=W, Y=Y, Z=Z, A1=A1, S=S, Qu=Qu, R=R, G=G,
               N=N, Q=Q)
    return out


def two_stage(V, A, qr_method="auto"):
    """Algorithm 1 with the second choice of P.  Returns (Q, R, S)."""
    o = two_stage_intermediates(V, A, qr_method=qr_method)
    return o["Q"], o["R"], o["S"]
