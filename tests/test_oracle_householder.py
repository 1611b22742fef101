"""Pins for the oracle's Householder QR (CPU only).

The oracle's column Householder is checked against LAPACK's Householder QR
(numpy.linalg.qr) after the nonnegative-diagonal normalization, which makes
the factorization unique for full-rank input; against the defining
properties (Q^*Q = I, R upper triangular with real nonnegative diagonal,
QR = X); and on rank-deficient special cases where the reflector must be
skipped (tau = 0).
"""

import numpy as np
import pytest

from oracle.householder import householder_qr, qr_pos, phase_normalize


def _rand(g, m, k, cplx):
    X = g.standard_normal((m, k))
    if cplx:
        X = X + 1j * g.standard_normal((m, k))
    return X


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("m,k", [(1, 1), (5, 3), (64, 64), (200, 17), (513, 40)])
def test_loop_matches_lapack(m, k, cplx):
    g = np.random.default_rng(7 + m + k)
    X = _rand(g, m, k, cplx)
    Q1, R1 = qr_pos(X, method="loop")
    Q2, R2 = qr_pos(X, method="lapack")
    assert np.allclose(Q1, Q2, atol=1e-12 * max(1, k))
    assert np.allclose(R1, R2, atol=1e-12 * np.abs(R2).max())


@pytest.mark.parametrize("cplx", [False, True])
def test_defining_properties(cplx):
    g = np.random.default_rng(3)
    X = _rand(g, 300, 12, cplx)
    Q, R = qr_pos(X, method="loop")
    assert np.allclose(np.tril(R, -1), 0)
    d = np.diag(R)
    assert np.all(np.imag(d) == 0) and np.all(np.real(d) >= 0)
    assert np.linalg.norm(np.conj(Q).T @ Q - np.eye(12), 2) < 1e-14
    assert np.linalg.norm(Q @ R - X, 2) / np.linalg.norm(X, 2) < 1e-14


def test_unnormalized_sign_convention():
    # xLARFG: beta = -sign(Re alpha) * norm, so R_00 < 0 when X_00 > 0
    X = np.array([[3.0, 1.0], [4.0, 2.0]])
    Q, R = householder_qr(X)
    assert R[0, 0] == pytest.approx(-5.0)
    Qn, Rn = phase_normalize(Q, R)
    assert Rn[0, 0] == pytest.approx(5.0)
    assert np.allclose(Qn @ Rn, X)


def test_zero_subcolumn_skips_reflection():
    # first column already upper triangular and positive: tau = 0, R_00 = X_00
    X = np.array([[2.0, 1.0], [0.0, 3.0], [0.0, 4.0]])
    Q, R = qr_pos(X, method="loop")
    assert R[0, 0] == 2.0
    assert np.allclose(Q[:, 0], [1, 0, 0])
    assert R[1, 1] == pytest.approx(5.0)


def test_rank_deficient_keeps_orthonormal_q():
    g = np.random.default_rng(11)
    B = g.standard_normal((100, 3))
    X = np.concatenate([B, B[:, :1] * 2.0, np.zeros((100, 1))], axis=1)
    Q, R = qr_pos(X, method="loop")
    assert np.linalg.norm(Q.T @ Q - np.eye(5), 2) < 1e-14
    assert np.linalg.norm(Q @ R - X, 2) < 1e-13 * np.linalg.norm(X, 2)
    assert abs(R[3, 3]) < 1e-13 and R[4, 4] == 0.0


def test_zero_matrix():
    Q, R = qr_pos(np.zeros((6, 3)), method="loop")
    assert np.allclose(R, 0)
    assert np.allclose(Q, np.eye(6)[:, :3])


def test_tiny_entries_no_underflow():
    # the 1e-30 entries of eq. (2): squares are 1e-60, well inside double range
    X = np.array([[1e-30, 0.0], [0.0, 1e-30], [0.0, 0.0]])
    Q, R = qr_pos(X, method="loop")
    assert np.allclose(np.diag(R), [1e-30, 1e-30], rtol=1e-15, atol=0)
    assert np.allclose(Q, np.eye(3)[:, :2])
