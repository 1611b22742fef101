"""Pins for the oracle's accuracy measures (CPU only): the chunked Gram against
a plain product, the 2-norms against LAPACK's SVD-based norm, and closed-form
values on constructed matrices."""

import numpy as np

from oracle import gram_chunked, spectral_norm_tall, orth_loss, orth_parts, rel_residual


def test_gram_chunked_matches_plain():
    g = np.random.default_rng(0)
    X = g.standard_normal((5000, 7)) + 1j * g.standard_normal((5000, 7))
    Y = g.standard_normal((5000, 3))
    assert np.allclose(gram_chunked(X, Y, chunk=333), np.conj(X).T @ Y)
    assert np.allclose(gram_chunked(X), np.conj(X).T @ X)


def test_spectral_norm_matches_svd():
    g = np.random.default_rng(1)
    X = g.standard_normal((3000, 9))
    assert abs(spectral_norm_tall(X) - np.linalg.norm(X, 2)) < 1e-12 * np.linalg.norm(X, 2)


def test_closed_form_losses():
    # V = [e1], Q = [cos t e1 + sin t e2]: ||[V,Q]^T[V,Q] - I||_2 = |cos t|
    t = 0.3
    V = np.array([[1.0], [0.0], [0.0]])
    Q = np.array([[np.cos(t)], [np.sin(t)], [0.0]])
    assert abs(orth_loss(V, Q) - abs(np.cos(t))) < 1e-15
    vq, qq = orth_parts(V, Q)
    assert abs(vq - abs(np.cos(t))) < 1e-15 and qq < 1e-15
    # residual of an exact decomposition is zero; of a perturbed one is known
    A = V @ np.array([[2.0]]) + Q @ np.array([[3.0]])
    assert rel_residual(V, A, Q, np.array([[3.0]]), np.array([[2.0]])) < 1e-15
    r = rel_residual(V, A, Q, np.array([[3.0]]), np.array([[2.5]]))
    assert abs(r - 0.5 / np.linalg.norm(A, 2)) < 1e-14
