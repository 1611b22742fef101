"""Pins for the oracle's block Householder-QR (Algorithm 4, §6.1).

  * exact arithmetic makes Algorithm 4 the QR factorization of the whole
    A = [A_1, ..., A_p] (Q^* Q = I, R upper triangular with nonnegative
    diagonal, unique for full-rank A), so on a well-conditioned A it must
    match LAPACK's Householder QR of A (library routine) after the sign fix;
  * with one block it is the Householder QR of A; with two blocks the second
    is exactly the two-stage method against the first block's Q;
  * stability on an extremely ill-conditioned stand-in for the s-step matrix
    of Example 5 (a monomial Krylov basis, cond ~ 7e17; the paper's matrices
    are not available): loss of orthogonality and residual at rounding level,
    the level of Table 5, for all three choices of P.
"""

import numpy as np
import pytest

import tho_workloads as W
from oracle import qr_pos, two_stage
from oracle.block_householder import block_bcgs2, block_householder


@pytest.mark.parametrize("cplx", [False, True])
def test_matches_lapack_qr_of_whole_matrix(cplx):
    g = np.random.default_rng(61)
    A = W.gaussian(g, (1500, 120), complex_=cplx)
    sizes = [10, 30, 7, 64, 9]
    Q, R = block_householder(A, sizes)
    Ql, Rl = qr_pos(A, method="lapack")
    assert np.max(np.abs(Q - Ql)) < 1e-12
    assert np.max(np.abs(R - Rl)) < 1e-12
    assert np.allclose(np.tril(R, -1), 0)


def test_one_and_two_blocks():
    g = np.random.default_rng(62)
    A = g.standard_normal((400, 20))
    Q1, R1 = block_householder(A, [20])
    Qh, Rh = qr_pos(A)
    assert np.array_equal(Q1, Qh) and np.array_equal(R1, Rh)
    Q2, R2 = block_householder(A, [12, 8])
    Qa, Ra = qr_pos(A[:, :12])
    Qb, Rb, Sb = two_stage(Qa, A[:, 12:])
    assert np.array_equal(Q2[:, :12], Qa) and np.array_equal(Q2[:, 12:], Qb)
    assert np.array_equal(R2[:12, 12:], Sb) and np.array_equal(R2[12:, 12:], Rb)


def krylov_standin(n=10000, p=50, k=10, seed=3):
    """Monomial block Krylov basis [X0, D X0, D^2 X0, ...] of a diagonal
    operator, columns normalized (input generation; cond ~ 7e17)."""
    g = np.random.default_rng(seed)
    d = np.linspace(0.1, 1.0, n)
    blocks = [g.standard_normal((n, k))]
    for _ in range(1, p):
        B = d[:, None] * blocks[-1]
        blocks.append(B / np.linalg.norm(B, axis=0))
    return np.concatenate(blocks, 1)


@pytest.mark.parametrize("choice", ["mlu", "qr", "polar"])
def test_stable_on_ill_conditioned_krylov_basis(choice):
    A = krylov_standin(n=3000, p=30, k=10)
    assert np.linalg.cond(A) > 1e15
    Q, R = block_householder(A, [10] * 30, p_choice=choice)
    kt = A.shape[1]
    loss = np.linalg.norm(Q.T @ Q - np.eye(kt), 2)
    res = np.linalg.norm(A - Q @ R, 2) / np.linalg.norm(A, 2)
    print(choice, "loss %.2e residual %.2e" % (loss, res))
    assert loss < 1e-13 and res < 1e-14
    Qb, Rb = block_bcgs2(A, [10] * 30)
    print("block BCGS2 loss %.2e" % np.linalg.norm(Qb.T @ Qb - np.eye(kt), 2))
