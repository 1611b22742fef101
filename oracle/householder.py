"""Column Householder QR with a nonnegative real diagonal of R (oracle).

Test infrastructure only (see ``oracle/__init__``).

Paper passages followed
  * The intra-block orthogonalization step is Householder-QR (§1, after
    eq. (1); the bottom-block QR of Algorithm 1).  Householder-QR satisfies Assumption 1
    (§4; Appendix B.1).
  * The second choice of P needs a QR factorization of the top k0 x k0 block
    of V whose R factor has nonnegative diagonal entries (§3.2, second
    choice; §6.1 and §6.2 use a QR variant producing such an R).

Reflector convention (the textbook / LAPACK one): for a column with pivot
alpha and subcolumn x, beta = -sign(Re alpha) * sqrt(|alpha|^2 + ||x||^2)
(sign(0) = +1), tau = (beta - alpha) / beta, u = [1; x / (alpha - beta)], and
H = I - tau u u^*, so that H^* [alpha; x] = [beta; 0].  When x = 0 and
alpha is real, tau = 0 (no reflection).  Q = H_1 H_2 ... H_k [I; 0].

Phase convention (the reading taken where the paper is silent on the sign of
diag(R) of the returned factors): every R returned by ``qr_pos`` has a real,
nonnegative diagonal and Q is scaled consistently; an exact zero diagonal
entry gets phase 1.
"""

import numpy as np

# Above this many matrix entries the oracle uses LAPACK's Householder QR
# (numpy.linalg.qr -> xGEQRF/xUNGQR) as a single library step instead of the
# column-by-column loop below; tests pin the two against each other.
_LOOP_LIMIT = 1 << 20


def _sign_re(a):
    """sign(Re a) with sign(0) = +1."""
    return -1.0 if np.real(a) < 0 else 1.0


def householder_qr(X):
    """Textbook column Householder QR of X (m x k, m >= k).

    Returns (Q, R) with Q (m x k) having orthonormal columns and R (k x k)
    upper triangular, diag(R) real with the xLARFG sign convention (not yet
    normalized).  Plain loops over columns; each step is one reflector.
    """
    X = np.array(X, dtype=np.result_type(X, np.float64), copy=True)
    m, k = X.shape
    if m < k:
        raise ValueError("householder_qr needs m >= k")
    taus = np.zeros(k, dtype=X.dtype)
    for j in range(k):
        alpha = X[j, j]
        x = X[j + 1:, j]
        xnorm2 = float(np.sum(np.abs(x) ** 2))
        if xnorm2 == 0.0 and np.imag(alpha) == 0.0:
            taus[j] = 0.0
            continue
        beta = -_sign_re(alpha) * np.sqrt(abs(alpha) ** 2 + xnorm2)
        tau = (beta - alpha) / beta
        v = x / (alpha - beta)
        X[j + 1:, j] = v
        X[j, j] = beta
        taus[j] = tau
        if j + 1 < k:
            # apply H_j^* = I - conj(tau) u u^* to the trailing columns
            u = np.concatenate(([1.0], v)).astype(X.dtype)
            w = np.conj(u) @ X[j:, j + 1:]
            X[j:, j + 1:] -= np.conj(tau) * np.outer(u, w)
    R = np.triu(X[:k, :k])
    # Q = H_1 ... H_k [I_k; 0], accumulated right to left
    Q = np.zeros((m, k), dtype=X.dtype)
    Q[:k, :k] = np.eye(k)
    for j in range(k - 1, -1, -1):
        if taus[j] == 0:
            continue
        u = np.concatenate(([1.0], X[j + 1:, j])).astype(X.dtype)
        w = np.conj(u) @ Q[j:, :]
        Q[j:, :] -= taus[j] * np.outer(u, w)
    return Q, R


def phase_normalize(Q, R):
    """Scale (Q, R) -> (Q D, D^* R) so that diag(R) is real and >= 0.

    D = diag(d_j), d_j = R_jj / |R_jj| (d_j = 1 when R_jj = 0).  Q R is
    unchanged and Q D keeps orthonormal columns.
    """
    diag = np.diag(R)
    mag = np.abs(diag)
    d = np.where(mag > 0, diag / np.where(mag > 0, mag, 1.0), 1.0)
    d = d.astype(np.result_type(R.dtype, np.float64))
    Qn = Q * d[None, :]
    Rn = np.conj(d)[:, None] * R
    # the diagonal is now real and nonnegative; store it exactly so
    Rn[np.arange(len(d)), np.arange(len(d))] = mag
    return Qn, Rn


def qr_pos(X, method="auto"):
    """Householder QR with nonnegative real diag(R) (xGEQRFP-style output).

    method: "loop" (textbook reflectors above), "lapack" (numpy.linalg.qr,
    itself a Householder QR, used as one library step) or "auto" (loop for
    small inputs).
    """
    X = np.asarray(X)
    if method == "auto":
        method = "loop" if X.size <= _LOOP_LIMIT else "lapack"
    if method == "loop":
        Q, R = householder_qr(X)
    elif method == "lapack":
        Q, R = np.linalg.qr(np.asarray(X, dtype=np.result_type(X, np.float64)),
                            mode="reduced")
    else:
        raise ValueError(method)
    return phase_normalize(Q, R)
