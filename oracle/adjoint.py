"""Reverse-mode gradient of the map the two-stage method computes (oracle,
real FP64 and complex128).

Test infrastructure only (see ``oracle/__init__``).

The paper is silent on differentiation.  Reading taken: differentiate exactly
the map (V, A) -> (Q, R, S) that ``two_stage.two_stage`` computes (second
choice of P, §3.1-§3.2), treating V and A as unconstrained matrices near an
orthonormal V.  For a scalar loss
    l = Re<G_Q, Q> + Re<G_R, R> + Re<G_S, S>,   <X, Y> = sum conj(X) * Y,
this module returns the gradients (V_bar, A_bar) defined by
dl = Re<V_bar, dV> + Re<A_bar, dA> (for real data the usual gradient; for
complex data the convention of PyTorch's complex autograd), by running the
adjoint of each step of the method in reverse order.  Both QR
factorizations (of V_top for P, and of the updated bottom block) have a
real positive diagonal, so each is the unique differentiable QR and uses the
thin-QR adjoint
    X = Q R, diag(R) > 0:  X_bar = (Q_bar + Q copyltu(M)) R^{-*},
    M = R R_bar^* - Q_bar^* Q,
    copyltu(M) = tril(M, -1) + tril(M, -1)^* + Re(diag(M)),
which for real data is the familiar tril(M) + tril(M, -1)^T.  Only the
upper triangle of R_bar (with the real part of its diagonal) and the lower
triangle of T_bar enter, since R and T are triangular with real diagonals.

``central_fd`` is the brute-force check: central differences of the forward
oracle along a (real or complex) direction.
"""

import numpy as np
from scipy.linalg import solve_triangular

from .two_stage import two_stage_intermediates


def _h(M):
    return np.conj(M).T


def _copyltu(M):
    L = np.tril(M, -1)
    out = L + _h(L)
    out[np.diag_indices_from(out)] = np.real(np.diag(M))
    return out


def _tri_bar(Rbar):
    """Upper triangle with real diagonal: the part of R_bar a triangular R
    with real diagonal can see."""
    U = np.triu(Rbar).astype(np.result_type(Rbar, np.float64), copy=True)
    U[np.diag_indices_from(U)] = np.real(np.diag(Rbar))
    return U


def qr_adjoint(Q, R, Qbar, Rbar):
    """Adjoint of the thin QR X = Q R with real positive diag(R)."""
    Rbar = _tri_bar(Rbar)
    M = R @ _h(Rbar) - _h(Qbar) @ Q
    B = Qbar + Q @ _copyltu(M)
    # B R^{-*}: solve X R^* = B, i.e. R X^* = B^*
    return _h(solve_triangular(R, _h(B), lower=False))


def two_stage_vjp(V, A, GQ, GR, GS=None):
    """(V_bar, A_bar) for l = Re<GQ,Q> + Re<GR,R> + Re<GS,S>."""
    V = np.asarray(V)
    A = np.asarray(A)
    dt = np.result_type(V, A, GQ, GR, np.float64)
    V = V.astype(dt, copy=False)
    A = A.astype(dt, copy=False)
    n, k0 = V.shape
    k = A.shape[1]
    o = two_stage_intermediates(V, A)
    P, R1, T, W, Z, A1, S, Qu, R, N = (o[x] for x in
                                      ("P", "R1", "T", "W", "Z", "A1", "S",
                                       "Qu", "R", "N"))
    Qbar = np.asarray(GQ, dtype=dt)
    Rbar = np.asarray(GR, dtype=dt)
    Sbar = (np.zeros((k0, k), dt) if GS is None else np.asarray(GS, dtype=dt))

    Wbar = np.zeros((n, k0), dt)
    Pbar = np.zeros((k0, k0), dt)
    Tbar = np.zeros((k0, k0), dt)
    Abar = np.zeros((n, k), dt)
    A1bar = np.zeros((n, k), dt)

    # formation of Q: Q = X - W N, N = T^{-1} G, G = W^* X, X = [0; Q_]
    X = np.zeros((n, k), dt)
    X[k0:] = Qu
    Xbar = Qbar.copy()
    Wbar -= Qbar @ _h(N)
    Nbar = -_h(W) @ Qbar
    if k0 > 0:
        Gbar = solve_triangular(_h(T), Nbar, lower=False)   # T^{-*} N_bar
    else:
        Gbar = np.zeros((0, k), dt)
    Tbar -= Gbar @ _h(N)
    Wbar += X @ _h(Gbar)
    Xbar += W @ Gbar
    Qubar = Xbar[k0:]

    # QR of the bottom block: A1_low = Q_ R
    A1bar[k0:] = qr_adjoint(Qu, R, Qubar, Rbar)

    # S = P^* A1_top
    Pbar += A1[:k0] @ _h(Sbar)
    A1bar[:k0] += P @ Sbar

    # update of A: A1 = A - W Z, Z = T^{-*} Y, Y = W^* A
    Abar += A1bar
    Wbar -= A1bar @ _h(Z)
    Zbar = -_h(W) @ A1bar
    if k0 > 0:
        Ybar = solve_triangular(T, Zbar, lower=True)      # T^{-1} Z_bar
    else:
        Ybar = np.zeros((0, k), dt)
    Tbar -= Z @ _h(Ybar)
    Wbar += A @ _h(Ybar)
    Abar += W @ Ybar

    # W = [P; 0] - V
    Vbar = -Wbar
    Pbar += Wbar[:k0]

    # choice of P and T: P = -Q1, T = I + R1^*, V_top = Q1 R1
    if k0 > 0:
        R1bar = _h(np.tril(Tbar))
        Q1bar = -Pbar
        Q1 = -P
        Vbar[:k0] += qr_adjoint(Q1, R1, Q1bar, R1bar)
    return Vbar, Abar


def loss_value(V, A, GQ, GR, GS=None):
    o = two_stage_intermediates(V, A)
    val = float(np.real(np.sum(np.conj(GQ) * o["Q"]) + np.sum(np.conj(GR) * np.triu(o["R"]))))
    if GS is not None:
        val += float(np.real(np.sum(np.conj(GS) * o["S"])))
    return val


def central_fd(V, A, GQ, GR, GS, dV, dA, h=1e-6):
    """Central difference of the loss along (dV, dA) with step h; equals
    Re<V_bar, dV> + Re<A_bar, dA> up to O(h^2)."""
    lp = loss_value(V + h * dV, A + h * dA, GQ, GR, GS)
    lm = loss_value(V - h * dV, A - h * dA, GQ, GR, GS)
    return (lp - lm) / (2.0 * h)
