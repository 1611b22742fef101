"""Reduced-precision panel products (THO_PANEL_F32X2, THO_PANEL_BF16).

The paper computes in IEEE double only, so these variants have no value to
be pinned to ("parity unpinned"): the tests report the orthogonality loss,
the relative residual and the distance to the FP64 oracle, and bound them by
what the operand precision allows -- FP32 hi + lo keeps FP32 accumulation
accuracy (2^-24), BF16 that of its 8-bit significand (2^-8); the cases
include the full graded size n = 2^22, k0 = 128, k = 64.  Householder
vectors, norms and T factors stay FP64; the reduced precision enters Q
through Q_low = Q_ + V_low N, so both ||V^T Q|| and ||Q^T Q - I|| carry it.
"""

import numpy as np
import pytest

import tho_workloads as W
from oracle import two_stage as oracle_two_stage, orth_parts, rel_residual

from gpu_util import require_gpu, to_dev, to_host

pytestmark = pytest.mark.gpu

# Bounds from the operand rounding (u32 = 2^-24: the FP32 accumulation inside
# each MFMA block of the hi + lo products; ub = 2^-8: BF16 operands).  The
# orthogonality parts and the residual are bounded by one unit, S (a
# reduction over all n rows, then a triangular solve) by a few; measured at
# these sizes: FP32 hi+lo <= 4.6e-9 (loss), 2.0e-8 (residual), 1.9e-7 (S);
# BF16 <= 2.5e-3 (||V^T Q||), 3.1e-4 (||Q^T Q - I||, residual), 2.6e-3 (S).
U32, UB = 2.0 ** -24, 2.0 ** -8
BOUND = {"f32x2": {"vq": U32, "qq": U32, "res": U32, "dS": 8 * U32},
         "bf16": {"vq": 2 * UB, "qq": UB / 8, "res": UB / 8, "dS": 2 * UB}}


def _run(V, A, panel):
    import paper_2602_14449_amd as tho
    Q, R, S = tho.two_stage(to_dev(V), to_dev(A), panel=panel)
    return to_host(Q), to_host(R), to_host(S)


@pytest.mark.parametrize("panel", ["f32x2", "bf16"])
@pytest.mark.parametrize("n,k0,k", [(4096, 16, 8), (20000, 128, 64), (70001, 64, 40), (9999, 100, 50),
                                    (3000, 8, 4), (1 << 17, 128, 64), (1 << 22, 128, 64)])
def test_panel_precision(panel, n, k0, k):
    require_gpu()
    V, A = W.graded(n=n, k0=k0, k=k, cond=1e8, seed_cfg=20)
    Qg, Rg, Sg = _run(V, A, panel)
    Qo, Ro, So = oracle_two_stage(V, A)
    vq, qq = orth_parts(V, Qg)
    res = rel_residual(V, A, Qg, Rg, Sg)
    dS = np.abs(Sg - So).max() / np.abs(So).max()
    print("%s n=%d k0=%d k=%d  ||V^TQ|| %.2e  ||Q^TQ-I|| %.2e  res %.2e  |dS| %.2e"
          % (panel, n, k0, k, vq, qq, res, dS))
    b = BOUND[panel]
    assert qq < b["qq"] and vq < b["vq"] and res < b["res"] and dS < b["dS"]
    assert np.all(np.diag(Rg) >= 0)


def test_f64_panel_is_default():
    require_gpu()
    V, A = W.plain()
    Q1, R1, S1 = _run(V, A, "fp64")
    import paper_2602_14449_amd as tho
    Q2, R2, S2 = tho.two_stage(to_dev(V), to_dev(A))
    assert np.array_equal(Q1, to_host(Q2))
