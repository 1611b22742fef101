"""Reverse-mode gradient of the map Algorithm 1 computes (oracle, real FP64).

Test infrastructure only (see ``oracle/__init__``).

The paper is silent on differentiation.  Reading taken: differentiate exactly
the map (V, A) -> (Q, R, S) that ``two_stage.two_stage`` computes (Algorithm 1
with the second choice of P, §3.1-§3.2), treating V and A as unconstrained
real matrices near an orthonormal V.  For a scalar loss
    l = <G_Q, Q> + <G_R, R> + <G_S, S>
this module returns (dl/dV, dl/dA) by running the adjoint of each line of
Algorithm 1 in reverse order.  Both QR factorizations (of V_top for P, and of
the updated bottom block) have a positive diagonal, so each is the unique
differentiable QR and uses the standard thin-QR adjoint
    X = Q R, diag(R) > 0:  X_bar = (Q_bar + Q copyltu(M)) R^{-T},
    M = R R_bar^T - Q_bar^T Q,  copyltu(M) = tril(M) + tril(M, -1)^T.
Only the upper triangle of R_bar and the lower triangle of T_bar enter, since
R and T are triangular.

``central_fd`` is the brute-force check: central differences of the forward
oracle along a direction.
"""

import numpy as np
from scipy.linalg import solve_triangular

from .two_stage import two_stage_intermediates


def _copyltu(M):
    return np.tril(M) + np.tril(M, -1).T


def qr_adjoint(Q, R, Qbar, Rbar):
    """Adjoint of the thin QR X = Q R with positive diag(R) (real)."""
    Rbar = np.triu(Rbar)
    M = R @ Rbar.T - Qbar.T @ Q
    B = Qbar + Q @ _copyltu(M)
    # B R^{-T}: solve X R^T = B, i.e. R X^T = B^T
    return solve_triangular(R, B.T, lower=False).T


def two_stage_vjp(V, A, GQ, GR, GS=None):
    """(dl/dV, dl/dA) for l = <GQ,Q> + <GR,R> + <GS,S> (real float64)."""
    V = np.asarray(V, dtype=np.float64)
    A = np.asarray(A, dtype=np.float64)
    n, k0 = V.shape
    k = A.shape[1]
    o = two_stage_intermediates(V, A)
    P, R1, T, W, Z, A1, S, Qu, R, N = (o[x] for x in
                                      ("P", "R1", "T", "W", "Z", "A1", "S",
                                       "Qu", "R", "N"))
    Qbar = np.asarray(GQ, dtype=np.float64)
    Rbar = np.asarray(GR, dtype=np.float64)
    Sbar = (np.zeros((k0, k)) if GS is None
            else np.asarray(GS, dtype=np.float64))

    Wbar = np.zeros((n, k0))
    Pbar = np.zeros((k0, k0))
    Tbar = np.zeros((k0, k0))
    Abar = np.zeros((n, k))
    A1bar = np.zeros((n, k))

    # formation of Q: Q = X - W N, N = T^{-1} G, G = W^T X, X = [0; Q_]
    X = np.zeros((n, k))
    X[k0:] = Qu
    Xbar = Qbar.copy()
    Wbar -= Qbar @ N.T
    Nbar = -W.T @ Qbar
    if k0 > 0:
        Gbar = solve_triangular(T.T, Nbar, lower=False)   # T^{-T} N_bar
    else:
        Gbar = np.zeros((0, k))
    Tbar -= Gbar @ N.T
    Wbar += X @ Gbar.T
    Xbar += W @ Gbar
    Qubar = Xbar[k0:]

    # QR of the bottom block: A1_low = Q_ R
    A1bar[k0:] = qr_adjoint(Qu, R, Qubar, Rbar)

    # S = P^T A1_top
    Pbar += A1[:k0] @ Sbar.T
    A1bar[:k0] += P @ Sbar

    # update of A: A1 = A - W Z, Z = T^{-T} Y, Y = W^T A
    Abar += A1bar
    Wbar -= A1bar @ Z.T
    Zbar = -W.T @ A1bar
    if k0 > 0:
        Ybar = solve_triangular(T, Zbar, lower=True)      # T^{-1} Z_bar
    else:
        Ybar = np.zeros((0, k))
    Tbar -= Z @ Ybar.T
    Wbar += A @ Ybar.T
    Abar += W @ Ybar

    # W = [P; 0] - V
    Vbar = -Wbar
    Pbar += Wbar[:k0]

    # choice of P and T: P = -Q1, T = I + R1^T, V_top = Q1 R1
    if k0 > 0:
        R1bar = np.triu(np.tril(Tbar).T)
        Q1bar = -Pbar
        Q1 = -P
        Vbar[:k0] += qr_adjoint(Q1, R1, Q1bar, R1bar)
    return Vbar, Abar


def loss_value(V, A, GQ, GR, GS=None):
    o = two_stage_intermediates(V, A)
    val = float(np.sum(GQ * o["Q"]) + np.sum(GR * np.triu(o["R"])))
    if GS is not None:
        val += float(np.sum(GS * o["S"]))
    return val


def central_fd(V, A, GQ, GR, GS, dV, dA, h=1e-6):
    """Central difference of the loss along (dV, dA) with step h."""
    lp = loss_value(V + h * dV, A + h * dA, GQ, GR, GS)
    lm = loss_value(V - h * dV, A - h * dA, GQ, GR, GS)
    return (lp - lm) / (2.0 * h)
