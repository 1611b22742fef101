"""GPU parity of the complex128 path (tho_two_stage, tho_bcgs, tho_hhqr_full
with THO_C128) against the CPU oracle in complex arithmetic.

Element-wise at 1e-10 on well-conditioned inputs (both sides return the
unique QR with real nonnegative diag(R)); on the complex workload
(A = V C + 1e-10 G, cond([V, A]) ~ 1e10) the invariants and the per-column
tolerance max(1e-10, 16 u kappa_j), and the loss pattern of the comparison
methods: two-stage and Householder QR at rounding level, BCGS(1,1) losing
orthogonality, BCGS(1,2) restoring it.
"""

import numpy as np
import pytest

import tho_workloads as W
from oracle import (two_stage as oracle_two_stage, bcgs as oracle_bcgs, hhqr_full as oracle_hhqr,
                    orth_loss, rel_residual)

from gpu_util import require_gpu, to_dev, to_host

pytestmark = pytest.mark.gpu


def _gpu(fn, V, A, *args):
    Q, R, S = fn(to_dev(V), to_dev(A), *args)
    return to_host(Q), to_host(R), to_host(S)


def _close(X, Y, tol):
    return np.abs(X - Y).max() < tol * max(1.0, np.abs(Y).max())


@pytest.mark.parametrize("n,k0,k", [(4096, 16, 8), (20000, 64, 32), (70001, 32, 17), (3000, 0, 9), (300, 5, 3),
                                    (96, 64, 32), (50000, 1, 1), (1 << 17, 64, 32)])
def test_complex_two_stage_parity(n, k0, k):
    require_gpu()
    import paper_2602_14449_amd as tho
    g = np.random.default_rng(1300 + n + k0 + k)
    V = W.orthonormal(g, n, k0, complex_=True)
    A = W.gaussian(g, (n, k), complex_=True)
    Qg, Rg, Sg = _gpu(tho.two_stage, V, A)
    Qo, Ro, So = oracle_two_stage(V, A)
    assert np.abs(Qg - Qo).max() < 1e-10, np.abs(Qg - Qo).max()
    assert _close(Rg, Ro, 1e-10)
    if k0:
        assert _close(Sg, So, 1e-10)
    assert np.all(np.abs(np.diag(Rg).imag) == 0) and np.all(np.diag(Rg).real >= 0)
    assert orth_loss(V, Qg) < 1e-12
    assert rel_residual(V, A, Qg, Rg, Sg) < 1e-12


@pytest.mark.parametrize("proj,rounds", [(1, 1), (2, 1), (1, 2)])
def test_complex_bcgs_parity(proj, rounds):
    require_gpu()
    import paper_2602_14449_amd as tho
    g = np.random.default_rng(77)
    n, k0, k = 30000, 64, 32
    V = W.orthonormal(g, n, k0, complex_=True)
    A = W.gaussian(g, (n, k), complex_=True)
    Qg, Rg, Sg = _gpu(tho.bcgs, V, A, proj, rounds)
    Qo, Ro, So = oracle_bcgs(V, A, proj=proj, rounds=rounds)
    assert np.abs(Qg - Qo).max() < 1e-10
    assert _close(Rg, Ro, 1e-10) and _close(Sg, So, 1e-10)


@pytest.mark.parametrize("n,k0,k", [(20000, 64, 32), (5000, 40, 7), (3000, 0, 5)])
def test_complex_hhqr_parity(n, k0, k):
    require_gpu()
    import paper_2602_14449_amd as tho
    g = np.random.default_rng(78 + n)
    V = W.orthonormal(g, n, k0, complex_=True)
    A = W.gaussian(g, (n, k), complex_=True)
    Qg, Rg, Sg = _gpu(tho.hhqr_full, V, A)
    Qo, Ro, So = oracle_hhqr(V, A)
    assert np.abs(Qg - Qo).max() < 1e-10
    assert _close(Rg, Ro, 1e-10)
    if k0:
        assert _close(Sg, So, 1e-10)


@pytest.mark.timeout(600)
def test_complex_workload_full_size():
    # the complex workload at its stated size: n = 2^20, k0 = 64, k = 32,
    # A = V C + 1e-10 G (cond([V, A]) ~ 1e10).  Two-stage Q, R, S element-wise
    # against the oracle, and the loss pattern of the comparison methods
    require_gpu()
    import paper_2602_14449_amd as tho
    print("complex workload n=2^20 k0=64 k=32", flush=True)
    V, A = W.complex_case(n=1 << 20)
    Qg, Rg, Sg = _gpu(tho.two_stage, V, A)
    Qo, Ro, So = oracle_two_stage(V, A)
    # per-column tolerance max(1e-10, 16 u kappa_j), kappa_j =
    # ||[V, A]||_2 / sigma_min([V, A_{:, :j+1}]) (~1e10 here: the rounding of
    # A - V V^H A relative to its 1e-10 size), from the R factor of [V, A]
    k0, k = V.shape[1], A.shape[1]
    RB = np.linalg.qr(np.concatenate([V, A], axis=1), mode="r")
    sv = [np.linalg.svd(RB[:k0 + j + 1, :k0 + j + 1], compute_uv=False)[-1] for j in range(k)]
    kap = np.linalg.svd(RB, compute_uv=False)[0] / np.maximum(sv, 1e-300)
    tolj = np.maximum(1e-10, 16 * 2.0 ** -53 * kap)
    err = np.max(np.abs(Qg - Qo), axis=0)
    print("kappa range %.2e .. %.2e, max|dQ| %.2e (max err/tol %.3f), max|dR| %.2e, max|dS| %.2e"
          % (kap.min(), kap.max(), err.max(), (err / tolj).max(), np.abs(Rg - Ro).max(), np.abs(Sg - So).max()),
          flush=True)
    assert np.all(err <= tolj), (err / tolj).max()
    # R is O(1e-10) here: two backward-stable computations of the R of
    # (I - V V^H) A agree to O(u ||A||) in absolute terms
    nA = np.linalg.norm(RB, 2)
    assert np.abs(Rg - Ro).max() < 1e3 * 2.0 ** -53 * nA
    assert _close(Sg, So, 1e-12)
    assert np.all(np.abs(np.diag(Rg).imag) == 0) and np.all(np.diag(Rg).real >= 0)
    res = {}
    for name, fn, args in [("two_stage", tho.two_stage, ()), ("hhqr", tho.hhqr_full, ()),
                           ("bcgs11", tho.bcgs, (1, 1)), ("bcgs12", tho.bcgs, (1, 2))]:
        Q, R, S = (Qg, Rg, Sg) if name == "two_stage" else _gpu(fn, V, A, *args)
        res[name] = (orth_loss(V, Q), rel_residual(V, A, Q, R, S))
        print(name, res[name], flush=True)
    assert res["two_stage"][0] < 1e-12 and res["two_stage"][1] < 1e-12
    assert res["hhqr"][0] < 1e-12 and res["hhqr"][1] < 1e-12
    assert res["bcgs11"][0] > 1e-9
    assert res["bcgs12"][0] < 1e-12
