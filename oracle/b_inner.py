"""Two-stage Householder-QR in a B-inner product (Algorithm 3, §5; Theorem 4)
-- oracle.

Test infrastructure only (see ``oracle/__init__``).

For a Hermitian positive definite B, V with V^* B V = I and any A, the result
is (Q, R, S) with
    [V, A] = [V, Q] [[I, S], [0, R]],   [V, Q]^* B [V, Q] = I      (the B form of eq. (4)),
R upper triangular with real nonnegative diagonal (the phase convention of
the rest of the oracle), unique for full-rank A.

``b_two_stage`` follows §5: an initial B-orthonormal basis U of k0 + k
columns from the Cholesky factor of B's leading principal submatrix,
U = [L_11^{-*}; 0]; P chosen from V^* B U_1 as in §3.2 (second choice:
U_1^* B V = Q1 R1, P = -Q1, T = I + R1^*); then the generalized Householder
transformation of Theorem 4, H = I - W T^{-1} W^* B with X = U_1 P, Y = V,
W = X - Y, maps X onto Y; A <- H^{-1} A = (I - W T^{-*} W^* B) A; the
components along U_1 P are removed by S = (U_1 P)^* B A, A <- A - U_1 P S;
the remainder is QR-factored in the B-inner product; Q = H Q_.

Reading (the paper is silent / refers elsewhere): the B-inner-product QR of
the remainder is delegated to [Shao2023]'s Householder-type algorithms, which
the paper does not state; here it is computed by the Cholesky transform,
B = L L^*:  L^* X = Q~ R (Householder QR),  Q_ = L^{-*} Q~, which gives the
same unique factorization in exact arithmetic (Q_^* B Q_ = Q~^* Q~ = I).

``b_two_stage_by_definition`` computes the same result from the plain
definition through the Cholesky transform of the whole problem:
L^* V is orthonormal, the Euclidean two-stage method on (L^* V, L^* A) gives
(Q~, R, S), and Q = L^{-*} Q~.
"""

import numpy as np
from scipy.linalg import cholesky, solve_triangular

from .householder import qr_pos
from .two_stage import two_stage


def _h(M):
    return np.conj(M).T


def _chol_lower(B):
    return cholesky(B, lower=True)


def b_qr(B, X):
    """QR of X in the B-inner product (Cholesky transform): X = Q R with
    Q^* B Q = I, diag(R) real >= 0."""
    L = _chol_lower(B)
    Qt, R = qr_pos(_h(L) @ X)
    return solve_triangular(_h(L), Qt, lower=False), R


def b_two_stage(B, V, A):
    """Algorithm 3 (second choice of P).  Returns (Q, R, S)."""
    B = np.asarray(B)
    V = np.asarray(V)
    A = np.asarray(A)
    dt = np.result_type(B, V, A, np.float64)
    n, k0 = V.shape
    k = A.shape[1]
    if n < k0 + k:
        raise ValueError("need n >= k0 + k")
    # initial B-orthonormal basis from the leading principal submatrix of B
    m = k0 + k
    L11 = _chol_lower(B[:m, :m])
    U = np.zeros((n, m), dt)
    U[:m, :] = solve_triangular(_h(L11), np.eye(m, dtype=dt), lower=False)
    U1 = U[:, :k0]
    BV = B @ V
    # P from V^* B U_1 (second choice): U_1^* B V = Q1 R1, P = -Q1
    if k0 > 0:
        Q1, R1 = qr_pos(_h(U1) @ BV, method="loop")
    else:
        Q1 = np.zeros((0, 0), dt)
        R1 = np.zeros((0, 0), dt)
    P = -Q1
    X = U1 @ P                               # U_1 <- U_1 P
    Wm = X - V
    T = np.eye(k0, dtype=dt) + _h(R1)        # = I - V^* B U_1 P
    BW = B @ Wm
    # A <- H^{-1} A = (I - W T^{-*} W^* B) A
    Z = solve_triangular(_h(T), _h(BW) @ A, lower=False) if k0 else np.zeros((0, k), dt)
    A1 = A - Wm @ Z
    # remove the components along U_1 P
    S = _h(X) @ (B @ A1)
    A2 = A1 - X @ S
    # QR of the remainder in the B-inner product
    Qu, R = b_qr(B, A2)
    # Q = H Q_ = (I - W T^{-1} W^* B) Q_
    N = solve_triangular(T, _h(BW) @ Qu, lower=True) if k0 else np.zeros((0, k), dt)
    Q = Qu - Wm @ N
    return Q, R, S


def b_two_stage_by_definition(B, V, A):
    """The same result through the Cholesky transform of the whole problem."""
    L = _chol_lower(np.asarray(B))
    Qt, R, S = two_stage(_h(L) @ V, _h(L) @ A)
    return solve_triangular(_h(L), Qt, lower=False), R, S


def b_generalized_householder(B, X, Y):
    """Theorem 4: H = I - W T^{-1} W^* B with W = X - Y, T = W^* B X."""
    Wm = X - Y
    T = _h(Wm) @ B @ X
    return np.eye(B.shape[0], dtype=np.result_type(B, X, Y)) - Wm @ np.linalg.solve(T, _h(Wm) @ B)
