"""Two-stage Householder orthogonalization (oracle), written from the
definitions of §3.1 and the choices of P of §3.2.

Test infrastructure only (see ``oracle/__init__``).

Definitions followed
  * §3.1, eq. (3): for X, Y with X^* X = Y^* Y, W = X - Y and T = W^* X
    nonsingular, H = I - W T^{-1} W^* is unitary with H X = Y.  Here
    X = [P; 0] for a unitary k0 x k0 matrix P and Y = V, so H = [V P^*, V_perp]
    and H [P; 0] = V.
  * Stage one applies H^* = I - W T^{-*} W^* to A: the top k0 rows of H^* A
    are P V^* A, the bottom n - k0 rows are V_perp^* A.  Hence S = V^* A is
    P^* times the top block.
  * Stage two QR-factors the bottom block, V_perp^* A = Q_ R, and sets
    Q = H [0; Q_]; then [V, A] = [V, Q] [[I, S], [0, R]] (eq. (4)).
  * P and the factored T come from ``choices.choose_p`` (first choice:
    modified LU; second: QR of V_top, the default and the paper's
    recommendation; third: polar decomposition).  For the second choice
    T = I + R1^* is the form analysed in Appendix B.2; it equals
    I - V_top^* P whenever Q1 is unitary (tested).

Readings taken where the paper is silent
  * Intra-block QR: column Householder with the nonnegative-diagonal phase
    convention (``householder.qr_pos``).
  * S is computed as P^* times the top block of H^* A (as in the method's
    statement), not as V^* A (they agree in exact arithmetic when V^* V = I).
  * n >= k0 + k is required; k0 = 0 reduces to qr_pos(A); k = 0 is a no-op.
"""

import numpy as np

from .choices import choose_p
from .householder import qr_pos


def _h(M):
    return np.conj(M).T


def apply_h_adjoint(Wm, Tf, B):
    """H^* B = B - W T^{-*} (W^* B).  Returns (H^* B, W^* B, T^{-*} W^* B)."""
    Y = _h(Wm) @ B
    Z = Tf.solve_h(Y)
    return B - Wm @ Z, Y, Z


def apply_h(Wm, Tf, B):
    """H B = B - W T^{-1} (W^* B).  Returns (H B, W^* B, T^{-1} W^* B)."""
    G = _h(Wm) @ B
    N = Tf.solve(G)
    return B - Wm @ N, G, N


def two_stage_intermediates(V, A, qr_method="auto", p_choice="qr"):
    """Run the two-stage method and return every intermediate.

    Returns a dict with P, T (explicit), Tf (factored T), W, Y (= W^* A),
    Z (= T^{-*} Y), A1 (= H^* A), S, Qu (Q_ of the bottom-block QR), R,
    G (= W^* [0; Q_]), N (= T^{-1} G) and Q; for the second choice also R1.
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
    # the generalized Householder transformation mapping [P; 0] onto V
    P, Tf = choose_p(V[:k0, :], p_choice)
    X = np.zeros((n, k0), dt)
    X[:k0, :] = P
    Wm = X - V
    # stage one: H^* A = [P V^* A; V_perp^* A]
    A1, Y, Z = apply_h_adjoint(Wm, Tf, A)
    S = _h(P) @ A1[:k0, :]
    # QR of V_perp^* A
    if k > 0:
        Qu, R = qr_pos(A1[k0:, :], method=qr_method)
    else:
        Qu = np.zeros((n - k0, 0), dt)
        R = np.zeros((0, 0), dt)
    # stage two: Q = H [0; Q_]
    Xq = np.zeros((n, k), dt)
    Xq[k0:, :] = Qu
    Q, G, N = apply_h(Wm, Tf, Xq)
    out = dict(P=P, T=Tf.T, Tf=Tf, W=Wm, Y=Y, Z=Z, A1=A1, S=S, Qu=Qu, R=R,
               G=G, N=N, Q=Q)
    out.update(Tf.parts)
    return out


def two_stage(V, A, qr_method="auto", p_choice="qr"):
    """The two-stage method; returns (Q, R, S)."""
    o = two_stage_intermediates(V, A, qr_method=qr_method, p_choice=p_choice)
    return o["Q"], o["R"], o["S"]
