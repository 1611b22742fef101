"""The three choices of the unitary P of Algorithm 1 and the matching T (oracle).

Test infrastructure only (see ``oracle/__init__``).

The generalized Householder transformation of §3.1 (eq. (3)) maps
X = [P; 0] onto Y = V with W = X - Y and T = W^* X = I - V_top^* P.  The
method never needs T itself, only solves with T and T^*; how those solves
are done depends on how P was chosen (§3.2, Appendix B.2):

  first choice   P diagonal, fixed while factoring P - V_top by the modified
                 LU of [BDGJKN2015] (Algorithm 2): P - V_top = L U, so
                 T = (P - V_top)^* P = U^* L^* P.
  second choice  V_top = Q1 R1 (Householder QR, diag(R1) >= 0), P = -Q1,
                 T = I + R1^*, lower triangular.
  third choice   polar decomposition V_top = Q2 M (M Hermitian positive
                 semidefinite, computed from an SVD as in §6.2), P = -Q2,
                 T = I + M, Hermitian positive definite: solves by Cholesky.

Every choice returns a ``TFactor`` with ``solve`` (T^{-1} B) and ``solve_h``
(T^{-*} B) and the explicit matrix T for the tests.
"""

import numpy as np
from scipy.linalg import cho_factor, cho_solve, solve_triangular

from .householder import qr_pos


def _h(M):
    return np.conj(M).T


def sign_re(mu):
    """sign(mu) of the first choice (§3.2): +1 when Re mu >= 0, else -1."""
    return 1.0 if np.real(mu) >= 0 else -1.0


def modified_lu(Z):
    """Modified LU factorization (Algorithm 2, §3.2) of a k x k matrix Z with
    ||Z||_2 <= 1.

    It is the LU factorization without pivoting of P - Z in which the
    diagonal unitary P is not known in advance: at elimination step i, once
    the Schur complement of the leading i x i block is formed, P_ii is set to
    -sign(z) where z is the (i, i) entry of the updated Z, so that the pivot
    P_ii - z has modulus at least one and no pivoting is needed.

    Returns (P, L, U): P diagonal with entries +-1, L unit lower triangular,
    U upper triangular, with P - Z = L U.
    """
    Zs = np.array(Z, dtype=np.result_type(Z, np.float64), copy=True)
    k = Zs.shape[0]
    if Zs.shape != (k, k):
        raise ValueError("modified_lu needs a square matrix")
    P = np.eye(k, dtype=Zs.dtype)
    L = np.eye(k, dtype=Zs.dtype)
    U = np.zeros((k, k), dtype=Zs.dtype)
    for i in range(k):
        # Zs[i:, i:] is the updated trailing block of Z (P - Zs[i:, i:] is
        # the Schur complement of P - Z); choose the pivot's sign first
        P[i, i] = -sign_re(Zs[i, i])
        U[i, i] = P[i, i] - Zs[i, i]
        U[i, i + 1:] = -Zs[i, i + 1:]
        L[i + 1:, i] = -Zs[i + 1:, i] / U[i, i]
        # Schur complement: (P - Z)_22 - L_21 U_12 = P_22 - (Z_22 + L_21 U_12)
        Zs[i + 1:, i + 1:] += np.outer(L[i + 1:, i], U[i, i + 1:])
    return P, L, U


def polar(M):
    """Polar decomposition M = Q2 H (Q2 unitary, H Hermitian positive
    semidefinite) of a square matrix from its SVD M = U_s diag(s) W_s^*:
    Q2 = U_s W_s^*, H = W_s diag(s) W_s^*.  The paper computes the polar
    factor of the third choice with an SVD (xGESDD, §6.2); numpy's SVD is the
    library step here.  H is returned exactly Hermitian."""
    M = np.asarray(M)
    if M.size == 0:
        return np.zeros_like(M, dtype=np.result_type(M, np.float64)), np.zeros_like(M, dtype=np.result_type(M, np.float64))
    Us, s, Wh = np.linalg.svd(M)
    Q2 = Us @ Wh
    H = _h(Wh) @ (s[:, None] * Wh)
    H = 0.5 * (H + _h(H))
    return Q2, H


class TFactor:
    """T of the generalized Householder transformation in the factored form
    its choice of P provides."""

    def __init__(self, choice, T, solve, solve_h, parts):
        self.choice = choice
        self.T = T
        self._solve = solve
        self._solve_h = solve_h
        self.parts = parts

    def solve(self, B):
        """T^{-1} B."""
        return self._solve(B)

    def solve_h(self, B):
        """T^{-*} B."""
        return self._solve_h(B)


def choose_p(Vtop, choice="qr"):
    """P and T for the top k0 x k0 block of V (§3.2).

    choice: "mlu" (first choice, Algorithm 2), "qr" (second choice) or
    "polar" (third choice).  Returns (P, TFactor).
    """
    Vtop = np.asarray(Vtop)
    dt = np.result_type(Vtop, np.float64)
    k0 = Vtop.shape[0]
    I = np.eye(k0, dtype=dt)
    if choice == "mlu":
        # P - V_top = L U  =>  T = (P - V_top)^* P = U^* L^* P
        P, L, U = modified_lu(Vtop)
        T = _h(L @ U) @ P

        def solve(B):      # T^{-1} = P^* L^{-*} U^{-*}
            y = solve_triangular(_h(U), B, lower=True)
            y = solve_triangular(_h(L), y, lower=False, unit_diagonal=True)
            return _h(P) @ y

        def solve_h(B):    # T^{-*} = U^{-1} L^{-1} P
            y = solve_triangular(L, P @ B, lower=True, unit_diagonal=True)
            return solve_triangular(U, y, lower=False)

        return P, TFactor("mlu", T, solve, solve_h, dict(L=L, U=U))
    if choice == "qr":
        # V_top = Q1 R1, diag(R1) >= 0;  P = -Q1;  T = I + R1^* (lower)
        if k0 > 0:
            Q1, R1 = qr_pos(Vtop, method="loop")
        else:
            Q1, R1 = np.zeros((0, 0), dt), np.zeros((0, 0), dt)
        P = -Q1
        T = I + _h(R1)

        def solve(B):
            return solve_triangular(T, B, lower=True) if k0 else np.zeros_like(B)

        def solve_h(B):
            return solve_triangular(_h(T), B, lower=False) if k0 else np.zeros_like(B)

        return P, TFactor("qr", T, solve, solve_h, dict(R1=R1))
    if choice == "polar":
        # V_top = Q2 M;  P = -Q2;  T = I + M (Hermitian positive definite)
        Q2, M = polar(Vtop)
        P = -Q2
        T = I + M
        if k0 > 0:
            cf = cho_factor(T, lower=True)

            def solve(B):
                return cho_solve(cf, B)
        else:
            def solve(B):
                return np.zeros_like(B)

        return P, TFactor("polar", T, solve, solve, dict(M=M))
    raise ValueError("unknown choice of P: %r" % (choice,))
