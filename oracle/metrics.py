"""Accuracy measures printed in the paper (oracle).

Test infrastructure only (see ``oracle/__init__``).

  * loss of orthogonality ||[V,Q]^*[V,Q] - I||_2 (Table 1, Example 1 of §6.1)
  * ||V^* Q||_2 and ||Q^* Q - I||_2 separately (Table 4)
  * relative residual ||A - V S - Q R||_2 / ||A||_2 (Table 4; Theorem 3)

Grams of very tall matrices are summed in FP64 over row chunks with a
pairwise (tree) sum of the chunk Grams, so that the measuring itself stays
far below the 1e-12 level being checked even at n = 2^22.
"""

import numpy as np

_CHUNK = 1024


def _h(M):
    return np.conj(M).T


def gram_chunked(X, Y=None, chunk=_CHUNK):
    """X^* Y (Y defaults to X) summed pairwise over row chunks of ``chunk``."""
    if Y is None:
        Y = X
    n = X.shape[0]
    parts = [_h(X[i:i + chunk]) @ Y[i:i + chunk] for i in range(0, n, chunk)]
    if not parts:
        return np.zeros((X.shape[1], Y.shape[1]),
                        dtype=np.result_type(X, Y, np.float64))
    while len(parts) > 1:
        nxt = [parts[i] + parts[i + 1] for i in range(0, len(parts) - 1, 2)]
        if len(parts) % 2:
            nxt.append(parts[-1])
        parts = nxt
    return parts[0]


def _herm_norm2(H):
    """2-norm of a Hermitian matrix = largest |eigenvalue|."""
    if H.size == 0:
        return 0.0
    H = 0.5 * (H + _h(H))
    return float(np.max(np.abs(np.linalg.eigvalsh(H))))


def spectral_norm_tall(X):
    """||X||_2 of a tall matrix via its chunked Gram."""
    if X.size == 0:
        return 0.0
    return float(np.sqrt(max(_herm_norm2(gram_chunked(X)), 0.0)))


def orth_loss(V, Q):
    """||[V, Q]^* [V, Q] - I||_2 (Table 1 / Example 1)."""
    B = np.concatenate([np.asarray(V), np.asarray(Q)], axis=1)
    G = gram_chunked(B)
    return _herm_norm2(G - np.eye(G.shape[0]))


def orth_parts(V, Q):
    """(||V^* Q||_2, ||Q^* Q - I||_2), the first two columns of Table 4."""
    VQ = gram_chunked(np.asarray(V), np.asarray(Q))
    QQ = gram_chunked(np.asarray(Q))
    vq = float(np.linalg.norm(VQ, 2)) if VQ.size else 0.0
    return vq, _herm_norm2(QQ - np.eye(QQ.shape[0]))


def rel_residual(V, A, Q, R, S, chunk=1 << 16):
    """||A - V S - Q R||_2 / ||A||_2 (Table 4, last column)."""
    A = np.asarray(A)
    n = A.shape[0]
    GE = None
    for i in range(0, n, chunk):
        E = A[i:i + chunk] - V[i:i + chunk] @ S - Q[i:i + chunk] @ R
        g = gram_chunked(E)
        GE = g if GE is None else GE + g
    na = spectral_norm_tall(A)
    if GE is None or na == 0.0:
        return 0.0
    return float(np.sqrt(max(_herm_norm2(GE), 0.0))) / na
