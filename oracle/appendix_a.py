"""The ill-conditioned modified-LU factor of eq. (6) and the construction of
Appendix A that realises it (oracle side, used to build Example 4's V).

Test infrastructure only (see ``oracle/__init__``).

eq. (6), §3.2: for k0 and alpha, the upper triangular U whose row i
(1-based) has diagonal 1 + alpha / sqrt(k0 - i + 1) and off-diagonal entries
-1 / sqrt(k0 - i + 1).  The paper states kappa_2(U) ~ 1.1e7 for k0 = 100,
alpha = 0.1.

Appendix A (Lemma A.1 and the theorem after it): modified LU applied to an
orthonormal V follows the trailing matrices of Householder QR applied to V
([BDGJKN2015, Lemma 6.2]); so V can be built by running Householder QR
backwards from the bottom-right corner, one row and one column at a time,
choosing each new first row freely (norm < 1).  Row i of U is fixed by the
first row r_i of the trailing matrix at step i: with P_ii = -sign(r_i[0]),
U_ii = P_ii - r_i[0] and U_i,j = -r_i[j - i] (Algorithm 2).
"""

import numpy as np


def badmlu_u(k0, alpha):
    """The matrix U of eq. (6)."""
    U = np.zeros((k0, k0))
    for i in range(k0):
        d = np.sqrt(k0 - i)
        U[i, i] = 1.0 + alpha / d
        U[i, i + 1:] = -1.0 / d
    return U


def schur_rows_for(U):
    """First rows r_i of the trailing matrices that make modified LU return U
    (Algorithm 2 read backwards).  Needs |U_ii| > 1 for every i."""
    k = U.shape[0]
    rows = []
    for i in range(k):
        u = U[i, i]
        if u > 1.0:
            r0 = 1.0 - u      # r0 < 0, so P_ii = +1 and U_ii = 1 - r0
        elif u < -1.0:
            r0 = -1.0 - u     # r0 > 0, so P_ii = -1 and U_ii = -1 - r0
        else:
            raise ValueError("modified LU pivots have modulus > 1 here")
        rows.append(np.concatenate(([r0], -U[i, i + 1:])))
    return rows


def _lemma_a1(Vs, b, g):
    """Lemma A.1: from Vs (m x c, orthonormal columns) and b (c + 1 entries,
    ||b|| < 1) build Vt ((m + 1) x (c + 1), orthonormal columns) with first
    row b^T whose first Householder step gives [[-sign(b_1), 0], [0, Vs]]."""
    m, c = Vs.shape
    sb = 1.0 if b[0] >= 0 else -1.0
    VH = np.zeros((m + 1, c + 1))
    VH[0, 0] = -sb
    VH[1:, 1:] = Vs
    # unit v orthogonal to the columns of VH (so v_1 = 0)
    v = np.zeros(m + 1)
    y = g.standard_normal(m)
    y -= Vs @ (Vs.T @ y)
    y -= Vs @ (Vs.T @ y)
    v[1:] = y / np.linalg.norm(y)
    nb2 = float(b @ b)
    if not nb2 < 1.0:
        raise ValueError("Lemma A.1 needs ||b|| < 1")
    x = np.sqrt(1.0 - nb2) * v + VH @ b
    # the reflector with H x = e_1: w = (x - e_1) / (x_1 - 1), tau = 1 - x_1
    # in exact arithmetic; tau is taken as 2 / (w^T w), which equals 1 - x_1
    # when ||x|| = 1 and keeps H orthogonal to rounding when ||x|| is off by
    # the orthogonality error of the previous steps (otherwise that error
    # would double with every step)
    w = (x - np.eye(m + 1)[0]) / (x[0] - 1.0)
    tau = 2.0 / float(w @ w)
    return VH - tau * np.outer(w, w @ VH)


def badmlu_v(n, U, g):
    """V (n x k0, orthonormal columns) such that the modified LU of its top
    k0 x k0 block returns U (Appendix A's construction)."""
    k0 = U.shape[0]
    rows = schur_rows_for(U)
    # bottom-right corner: one column [r_k0[0]; x], a unit vector
    x = g.standard_normal(n - k0)
    r0 = rows[-1][0]
    Vs = np.concatenate(([r0], np.sqrt(1.0 - r0 * r0) * x / np.linalg.norm(x)))[:, None]
    for i in range(k0 - 2, -1, -1):
        Vs = _lemma_a1(Vs, rows[i], g)
    return np.ascontiguousarray(Vs)
