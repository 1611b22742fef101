"""Block Householder-QR of a sequence of blocks (Algorithm 4, §6.1) and the
block BCGS2 baseline it is compared with (Table 5) -- oracle.

Test infrastructure only (see ``oracle/__init__``).

Algorithm 4 factors A = [A_1, ..., A_p] block by block, as block Krylov
methods produce the blocks: A_1 = Q_1 R_1 by Householder QR; then for each
later block the generalized Householder transformation H of §3.1 is built
from the basis found so far, V = [Q_1, ..., Q_{i-1}], and the two-stage
method (``two_stage``) gives Q_i, the off-diagonal block S_i = V^* A_i and
the diagonal block R_i of R.  The result is A = Q R with Q^* Q = I and R
upper triangular (nonnegative diagonal, the phase convention of the rest of
the oracle).

Block BCGS2: for each block, two rounds of (project against all earlier
columns, Householder QR), the BCGS-with-reorthogonalization pattern of
Table 1 applied block by block.
"""

import numpy as np

from .baselines import bcgs
from .householder import qr_pos
from .two_stage import two_stage


def _split(k_total, block_sizes):
    if sum(block_sizes) != k_total or any(b <= 0 for b in block_sizes):
        raise ValueError("block sizes must be positive and add up to the number of columns")
    c = np.concatenate(([0], np.cumsum(block_sizes)))
    return [(int(c[i]), int(c[i + 1])) for i in range(len(block_sizes))]


def block_householder(A, block_sizes, p_choice="qr"):
    """Algorithm 4 on the column blocks of A.  Returns (Q, R)."""
    A = np.asarray(A)
    dt = np.result_type(A, np.float64)
    n, kt = A.shape
    if n < kt:
        raise ValueError("need n >= total number of columns")
    Q = np.zeros((n, kt), dt)
    R = np.zeros((kt, kt), dt)
    for i, (c0, c1) in enumerate(_split(kt, block_sizes)):
        if i == 0:
            Qi, Ri = qr_pos(A[:, c0:c1])
            Si = np.zeros((0, c1 - c0), dt)
        else:
            Qi, Ri, Si = two_stage(Q[:, :c0], A[:, c0:c1], p_choice=p_choice)
        Q[:, c0:c1] = Qi
        R[:c0, c0:c1] = Si
        R[c0:c1, c0:c1] = Ri
    return Q, R


def block_bcgs2(A, block_sizes):
    """Block BCGS2 baseline (Table 5).  Returns (Q, R)."""
    A = np.asarray(A)
    dt = np.result_type(A, np.float64)
    n, kt = A.shape
    Q = np.zeros((n, kt), dt)
    R = np.zeros((kt, kt), dt)
    for i, (c0, c1) in enumerate(_split(kt, block_sizes)):
        Qi, Ri, Si = bcgs(Q[:, :c0], A[:, c0:c1], proj=1, rounds=2)
        Q[:, c0:c1] = Qi
        R[:c0, c0:c1] = Si
        R[c0:c1, c0:c1] = Ri
    return Q, R
