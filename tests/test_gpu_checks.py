"""The numerical-condition channel of tho_two_stage on the GPU: the info word
(tho_get_info) after THO_CHECK_FINITE and THO_CHECK_VORTH.

Expected values come from the inputs' construction (a NaN or infinity
planted on the host at a chosen place, a V perturbed by 1e-6 so that
||V^T V - I||_F ~ 1e-5 > 1e-10), not from the GPU."""

import ctypes

import numpy as np
import pytest
import torch

import tho_workloads as W
from gpu_util import require_gpu, to_dev

pytestmark = pytest.mark.gpu


def _run(V, A, **flags):
    import paper_2602_14449_amd as tho
    Vd, Ad = to_dev(V), to_dev(A)
    nb = tho.workspace_bytes(V.shape[0], V.shape[1], A.shape[1], dtype=Ad.dtype, **flags)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    Q, R, S = tho.two_stage(Vd, Ad, workspace=ws, **flags)
    return tho.get_info(ws), Q, R, S


def _inputs(n=20000, k0=32, k=16, seed=91, cplx=False):
    g = np.random.default_rng(seed)
    V = W.orthonormal(g, n, k0, complex_=cplx)
    A = np.ascontiguousarray(W.gaussian(g, (n, k), complex_=cplx))
    return V, A


@pytest.mark.parametrize("where", ["A_top", "A_low", "V_top", "V_low", "A_inf", "V_inf"])
def test_nonfinite_input_sets_info_1(where):
    require_gpu()
    V, A = _inputs()
    val = np.inf if where.endswith("inf") else np.nan
    (A if where[0] == "A" else V)[{"A_top": 3, "V_top": 5}.get(where, 12345), 7] = val
    print("case", where, flush=True)
    info, Q, R, S = _run(V, A, check_finite=True)
    assert info == 1
    info0, *_ = _run(V, A)                   # no check requested: nothing reported
    assert info0 == 0


def test_nonfinite_k0_zero():
    require_gpu()
    V, A = _inputs(k0=0)
    A[777, 3] = np.nan
    assert _run(V, A, check_finite=True)[0] == 1


def test_clean_inputs_report_nothing():
    require_gpu()
    for k0 in (0, 1, 32, 128):
        V, A = _inputs(k0=k0, k=64 if k0 == 128 else 16)
        info, Q, R, S = _run(V, A, check_finite=True, check_vorth=True)
        assert info == 0, k0
        assert torch.isfinite(Q).all()


def test_perturbed_v_sets_info_3():
    require_gpu()
    V, A = _inputs(k0=100, k=20)
    g = np.random.default_rng(5)
    Vp = V + 1e-6 * g.standard_normal(V.shape)
    dev = np.linalg.norm(Vp.T @ Vp - np.eye(100))
    assert dev > 1e-8
    assert _run(Vp, A, check_vorth=True)[0] == 3
    assert _run(Vp, A)[0] == 0
    assert _run(V, A, check_vorth=True)[0] == 0
    # both conditions: the smaller code wins
    Vp[10, 3] = np.nan
    assert _run(Vp, A, check_vorth=True, check_finite=True)[0] == 1


def test_complex_checks():
    require_gpu()
    V, A = _inputs(n=30000, k0=24, k=8, cplx=True)
    assert _run(V, A, check_finite=True, check_vorth=True)[0] == 0
    g = np.random.default_rng(6)
    Vp = V + 1e-6 * (g.standard_normal(V.shape) + 1j * g.standard_normal(V.shape))
    assert _run(Vp, A, check_vorth=True)[0] == 3
    A2 = A.copy()
    A2[100, 2] = complex(0.0, np.nan)
    assert _run(V, A2, check_finite=True)[0] == 1


def test_noalloc_info_word():
    require_gpu()
    from paper_2602_14449_amd import _lib as L
    import paper_2602_14449_amd as tho
    V, A = _inputs(n=10000, k0=16, k=8)
    A[50, 1] = np.nan
    Vd, Ad = to_dev(V), to_dev(A)
    Q = torch.empty((10000, 8), dtype=torch.float64, device="cuda")
    R = torch.empty((8, 8), dtype=torch.float64, device="cuda")
    S = torch.empty((16, 8), dtype=torch.float64, device="cuda")
    o = L.Opts()
    o.flags = L.CHECK_FINITE
    rc = L.tho_two_stage_noalloc(0, 10000, 16, 8, Vd.data_ptr(), 16, Ad.data_ptr(), 8, Q.data_ptr(), 8,
                                 R.data_ptr(), 8, S.data_ptr(), 8, ctypes.byref(o),
                                 torch.cuda.current_stream().cuda_stream)
    L.check(rc, "tho_two_stage_noalloc")
    assert tho.get_info(None) == 1
