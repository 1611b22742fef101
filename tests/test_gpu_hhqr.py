"""GPU parity of the full Householder QR of [V, A] (tho_hhqr_full) against
the CPU oracle (Householder QR of the concatenated matrix, nonnegative
diag R_B; Q = Q_B[:, k0:], R = R_B[k0:, k0:], S = R_B[:k0, k0:])."""

import numpy as np
import pytest

import tho_workloads as W
from oracle import hhqr_full as oracle_hhqr, orth_loss, rel_residual

from gpu_util import require_gpu, to_dev, to_host

pytestmark = pytest.mark.gpu


def _run(V, A):
    import paper_2602_14449_amd as tho
    Q, R, S = tho.hhqr_full(to_dev(V), to_dev(A))
    return to_host(Q), to_host(R), to_host(S)


@pytest.mark.parametrize("n,k0,k", [(4096, 16, 8), (20000, 128, 64), (9999, 100, 50), (70001, 64, 40),
                                    (3000, 0, 12), (300, 65, 3), (192, 128, 64)])
def test_hhqr_parity(n, k0, k):
    require_gpu()
    g = np.random.default_rng(900 + n + k0 + k)
    V = W.orthonormal(g, n, k0)
    A = g.standard_normal((n, k))
    Qg, Rg, Sg = _run(V, A)
    Qo, Ro, So = oracle_hhqr(V, A)
    assert np.abs(Qg - Qo).max() < 1e-10
    assert np.abs(Rg - Ro).max() < 1e-10 * max(1.0, np.abs(Ro).max())
    if k0:
        assert np.abs(Sg - So).max() < 1e-10 * max(1.0, np.abs(So).max())
    assert orth_loss(V, Qg) < 1e-12
    assert rel_residual(V, A, Qg, Rg, Sg) < 1e-12


def test_hhqr_does_not_assume_orthonormal_v():
    # a Gaussian (non-orthonormal) V: the factorization of [V, A] is still
    # the oracle's, and Q_B's last columns are orthonormal
    require_gpu()
    g = np.random.default_rng(77)
    n, k0, k = 20000, 96, 32
    V = g.standard_normal((n, k0))
    A = g.standard_normal((n, k))
    Qg, Rg, Sg = _run(V, A)
    Qo, Ro, So = oracle_hhqr(V, A)
    scale = max(np.abs(Ro).max(), np.abs(So).max())
    assert np.abs(Qg - Qo).max() < 1e-10
    assert np.abs(Rg - Ro).max() < 1e-10 * scale
    assert np.abs(Sg - So).max() < 1e-10 * scale
    assert np.abs(Qg.T @ Qg - np.eye(k)).max() < 1e-13


def test_hhqr_ill_conditioned():
    # A = V C + 1e-10 G: cond([V, A]) ~ 1e10; Householder keeps loss at
    # rounding level
    require_gpu()
    g = np.random.default_rng(10)
    n, k0, k = 1 << 16, 64, 32
    V = W.orthonormal(g, n, k0)
    A = V @ g.standard_normal((k0, k)) + 1e-10 * g.standard_normal((n, k))
    Qg, Rg, Sg = _run(V, A)
    assert orth_loss(V, Qg) < 1e-13
    assert rel_residual(V, A, Qg, Rg, Sg) < 1e-13
