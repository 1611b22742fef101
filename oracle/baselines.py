"""The two comparison methods of the paper (oracle).

Test infrastructure only (see ``oracle/__init__``).

hhqr_full
  The naive approach named at the start of §3: Householder-QR of the whole
  n x (k0 + k) matrix [V, A], ignoring that V is orthonormal.  With the
  nonnegative-diagonal convention, [V, A] = Q_B R_B gives the same
  decomposition as eq. (4): Q = Q_B[:, k0:], R = R_B[k0:, k0:],
  S = R_B[:k0, k0:] (and R_B[:k0, :k0] ~ I when V^* V = I).

bcgs
  The BCGS framework of eq. (1): (BQR-1) A <- A - V V^* A, (BQR-2) A = Q R,
  with the repetition patterns of Table 1.  Reading (the paper lists the
  patterns but not how S and R accumulate): a run is ``rounds`` rounds, each
  doing ``proj`` times (BQR-1) followed by one (BQR-2).  Round r >= 2 starts
  from the previous round's Q.  With S_r the sum of the V^* X products of
  round r and R_r its triangular factor,
      A = V (S_1 + S_2 R_1 + S_3 R_2 R_1 + ...) + Q_r (R_r ... R_1).
  Table 1 rows map to (proj, rounds) = (1,1), (2,1), (1,2), (3,1), (1,3).
  The intra-block QR is Householder (``qr_pos``).
"""

import numpy as np

from .householder import qr_pos


def _h(M):
    return np.conj(M).T


def hhqr_full(V, A, qr_method="auto"):
    """Householder QR of [V, A]; returns (Q, R, S) in the layout of eq. (4)."""
    V = np.asarray(V)
    A = np.asarray(A)
    dt = np.result_type(V, A, np.float64)
    k0 = V.shape[1]
    B = np.concatenate([V.astype(dt), A.astype(dt)], axis=1)
    QB, RB = qr_pos(B, method=qr_method)
    return QB[:, k0:], RB[k0:, k0:], RB[:k0, k0:]


def bcgs(V, A, proj=1, rounds=1, qr_method="auto"):
    """BCGS with ``proj`` projections per round and ``rounds`` rounds.

    Returns (Q, R, S) with A ~ V S + Q R.
    """
    V = np.asarray(V)
    A = np.asarray(A)
    dt = np.result_type(V, A, np.float64)
    V = V.astype(dt, copy=False)
    X = A.astype(dt, copy=True)
    k0 = V.shape[1]
    k = A.shape[1]
    S = np.zeros((k0, k), dt)
    Rtot = np.eye(k, dtype=dt)
    for _ in range(rounds):
        Sr = np.zeros((k0, k), dt)
        for _ in range(proj):
            C = _h(V) @ X          # (BQR-1)
            X = X - V @ C
            Sr = Sr + C
        X, Rr = qr_pos(X, method=qr_method)  # (BQR-2)
        S = S + Sr @ Rtot
        Rtot = Rr @ Rtot
    return X, Rtot, S
