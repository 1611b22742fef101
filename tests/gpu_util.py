"""Helpers for the GPU parity tests (test infrastructure)."""

import numpy as np
import pytest
import torch


def require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def to_host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def col_errors(Q, Qref):
    """Per-column max abs difference after unit-phase alignment of Q to Qref."""
    d = np.sum(np.conj(Q) * Qref, axis=0)
    ph = np.where(np.abs(d) > 0, d / np.where(np.abs(d) > 0, np.abs(d), 1), 1)
    return np.max(np.abs(Q * ph[None, :] - Qref), axis=0) if Q.size else np.zeros(0)


def gpu_gram(X, Y=None, chunk=1 << 16):
    """FP64 X^T Y on the GPU, summed over row chunks (for large-size checks)."""
    if Y is None:
        Y = X
    out = None
    for i in range(0, X.shape[0], chunk):
        g = X[i:i + chunk].conj().transpose(0, 1).contiguous() @ Y[i:i + chunk]
        out = g if out is None else out + g
    return out


def herm_norm2(H):
    H = 0.5 * (H + H.conj().T)
    return float(np.max(np.abs(np.linalg.eigvalsh(H)))) if H.size else 0.0
