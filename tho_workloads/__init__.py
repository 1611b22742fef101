"""Seeded synthetic inputs shared by the tests, the bench and the oracle checks.

This module holds input generation only (random matrices with the shapes and
conditioning of the workloads) and none of the orthogonalization arithmetic.
Both the CPU oracle and the GPU library consume its outputs; neither is
imported here.

Workloads (each stands in for data the paper itself does not ship; the
paper's experiments use MATLAB ``randn`` matrices and LAPACK ``xLAGGE``
matrices with a prescribed condition number, §6.1-§6.2):

  plain     real, n=4096, k0=16, k=8: V = Q factor of a Gaussian n x k0,
            A Gaussian n x k
  example2  the 4 x 2 worked example of eq. (2) (V with +-sqrt(2)/2 entries,
            A with 1e-30 entries), exactly as printed
  complex   complex128, n=2^20, k0=64, k=32: V = Q factor of a complex
            Gaussian, A = V C + 1e-10 G, so [V, A] has condition ~1e10
  graded    real, n=2^22, k0=128, k=64: V = Q factor of a Gaussian,
            A = X diag(s) Y^T with X, Y orthonormal Gaussian-derived and s
            log-spaced from 1 to 1e-8 (condition 1e8)
  batched   4096 independent real instances, n ~ U{2048..65536},
            k0 ~ U{8,16,32,64}, k ~ U{4,8,16}
  grad      real, n=2^20, k0=64, k=32, with Gaussian G_Q, G_R loss weights

Seeds: numpy Generator(PCG64(260214449 + cfg)); batched instance j uses the
j-th child of SeedSequence(260214449).  Complex Gaussian entries are
(N(0,1) + i N(0,1)) / sqrt(2).
"""

import numpy as np

BASE_SEED = 260214449


def rng(cfg):
    return np.random.Generator(np.random.PCG64(BASE_SEED + cfg))


def gaussian(g, shape, complex_=False):
    if complex_:
        re = g.standard_normal(shape)
        im = g.standard_normal(shape)
        return (re + 1j * im) / np.sqrt(2.0)
    return g.standard_normal(shape)


def orthonormal(g, n, k, complex_=False):
    """Q factor (n x k) of a Gaussian matrix (LAPACK QR; input generation)."""
    if k == 0:
        return np.zeros((n, 0), dtype=np.complex128 if complex_ else np.float64)
    q, _ = np.linalg.qr(gaussian(g, (n, k), complex_), mode="reduced")
    return np.ascontiguousarray(q)


def example2():
    """The 4 x 2 matrices of eq. (2)."""
    s = np.sqrt(2.0)
    V = 0.5 * np.array([[s, s], [-s, s], [0.0, 0.0], [0.0, 0.0]])
    A = np.array([[1.0, 1.0], [1.0, 1.0], [1e-30, 0.0], [0.0, 1e-30]])
    return V, A


def plain(n=4096, k0=16, k=8, seed_cfg=1):
    g = rng(seed_cfg)
    V = orthonormal(g, n, k0)
    A = np.ascontiguousarray(gaussian(g, (n, k)))
    return V, A


def complex_case(n=1 << 20, k0=64, k=32, eps=1e-10, seed_cfg=2):
    g = rng(seed_cfg)
    V = orthonormal(g, n, k0, complex_=True)
    C = gaussian(g, (k0, k), complex_=True)
    G = gaussian(g, (n, k), complex_=True)
    A = np.ascontiguousarray(V @ C + eps * G)
    return V, A


def graded(n=1 << 22, k0=128, k=64, cond=1e8, seed_cfg=3):
    g = rng(seed_cfg)
    V = orthonormal(g, n, k0)
    X = orthonormal(g, n, k)
    Y = orthonormal(g, k, k)
    if k > 1:
        s = 10.0 ** (-np.log10(cond) * np.arange(k) / (k - 1))
    else:
        s = np.ones(k)
    A = np.ascontiguousarray((X * s[None, :]) @ Y.T)
    return V, A


def batched_shapes(count=4096, seed_cfg=4):
    """(n, k0, k) per instance for the batched workload."""
    ss = np.random.SeedSequence(BASE_SEED)
    kids = ss.spawn(count)
    shapes = []
    for c in kids:
        g = np.random.Generator(np.random.PCG64(c))
        n = int(g.integers(2048, 65536, endpoint=True))
        k0 = int(g.choice([8, 16, 32, 64]))
        k = int(g.choice([4, 8, 16]))
        shapes.append((n, k0, k))
    return shapes


def batched_instance(j, count=4096):
    """Inputs of batched instance j (same stream as ``batched_shapes``)."""
    ss = np.random.SeedSequence(BASE_SEED)
    c = ss.spawn(count)[j]
    g = np.random.Generator(np.random.PCG64(c))
    n = int(g.integers(2048, 65536, endpoint=True))
    k0 = int(g.choice([8, 16, 32, 64]))
    k = int(g.choice([4, 8, 16]))
    V = orthonormal(g, n, k0)
    A = np.ascontiguousarray(gaussian(g, (n, k)))
    return V, A


def grad_case(n=1 << 20, k0=64, k=32, seed_cfg=5):
    g = rng(seed_cfg)
    V = orthonormal(g, n, k0)
    A = np.ascontiguousarray(gaussian(g, (n, k)))
    GQ = np.ascontiguousarray(gaussian(g, (n, k)))
    GR = np.ascontiguousarray(gaussian(g, (k, k)))
    return V, A, GQ, GR


def batched_gpu(count=4096, device="cuda", seed_cfg=4):
    """The batched workload generated on a GPU with torch (input generation
    only): the shapes of ``batched_shapes``, Gaussian A, and V the Q factor of
    a Gaussian matrix by two rounds of Cholesky QR (orthonormal to ~1e-15 for
    these well-conditioned matrices).  Returns a list of (V, A) tensors."""
    import torch
    shapes = batched_shapes(count, seed_cfg)
    g = torch.Generator(device=device).manual_seed(BASE_SEED + seed_cfg)
    out = []
    for (n, k0, k) in shapes:
        X = torch.randn(n, k0, dtype=torch.float64, device=device, generator=g)
        for _ in range(2):
            G = X.T.contiguous() @ X
            Lc = torch.linalg.cholesky(G)
            X = torch.linalg.solve_triangular(Lc, X.T.contiguous(), upper=False).T.contiguous()
        A = torch.randn(n, k, dtype=torch.float64, device=device, generator=g)
        out.append((X, A))
    return out
