"""Argument checks of the Python binding that need no GPU: caller-supplied
output tensors must match the shapes the C ABI writes, and inputs whose rows
overlap in memory (expanded views) are rejected before any pointer reaches
the library."""

import pytest
import torch

from paper_2602_14449_amd import api


def test_expanded_input_rejected():
    n, k0, k = 64, 4, 3
    V = torch.zeros(n, k0, dtype=torch.float64)
    A = torch.randn(1, k, dtype=torch.float64).expand(n, k)
    with pytest.raises(ValueError, match="overlapping rows"):
        api._check_inputs(V, A)
    with pytest.raises(ValueError, match="overlapping rows"):
        api._check_inputs(torch.zeros(1, k0, dtype=torch.float64).expand(n, k0),
                          torch.zeros(n, k, dtype=torch.float64))


def test_cpu_inputs_rejected():
    with pytest.raises(ValueError, match="GPU"):
        api._check_inputs(torch.zeros(8, 2, dtype=torch.float64), torch.zeros(8, 2, dtype=torch.float64))


def test_dtype_and_rank_rejected():
    with pytest.raises(TypeError):
        api._check_inputs(torch.zeros(8, 2, dtype=torch.float32), torch.zeros(8, 2, dtype=torch.float32))
    with pytest.raises(ValueError):
        api._check_inputs(torch.zeros(8, dtype=torch.float64), torch.zeros(8, 2, dtype=torch.float64))


@pytest.mark.parametrize("which,shape,dtype", [
    (0, (63, 3), torch.float64),    # Q too short
    (1, (3, 2), torch.float64),     # R too small
    (2, (4, 4), torch.float64),     # S wrong width
    (0, (64, 3), torch.float32),    # wrong dtype
])
def test_wrong_out_rejected(which, shape, dtype):
    n, k0, k = 64, 4, 3
    like = torch.zeros(n, k, dtype=torch.float64)
    good = [torch.zeros(n, k, dtype=torch.float64), torch.zeros(k, k, dtype=torch.float64),
            torch.zeros(k0, k, dtype=torch.float64)]
    good[which] = torch.zeros(*shape, dtype=dtype)
    with pytest.raises((ValueError, TypeError)):
        api._outputs(tuple(good), n, k0, k, like)


def test_expanded_out_rejected():
    n, k0, k = 64, 4, 3
    like = torch.zeros(n, k, dtype=torch.float64)
    Q = torch.zeros(1, k, dtype=torch.float64).expand(n, k)
    with pytest.raises(ValueError, match="overlapping rows"):
        api._outputs((Q, torch.zeros(k, k, dtype=torch.float64), torch.zeros(k0, k, dtype=torch.float64)),
                     n, k0, k, like)


def test_good_out_accepted():
    n, k0, k = 64, 4, 3
    like = torch.zeros(n, k, dtype=torch.float64)
    out = (torch.zeros(n, k, dtype=torch.float64), torch.zeros(k, k, dtype=torch.float64),
           torch.zeros(k0, k, dtype=torch.float64))
    assert api._outputs(out, n, k0, k, like) == out


def test_workspace_must_be_bytes_on_device():
    with pytest.raises(ValueError):
        api._workspace(100, torch.zeros(100, dtype=torch.float64), torch.device("cpu"))
    ws = torch.zeros(128, dtype=torch.uint8)
    assert api._workspace(100, ws, torch.device("cpu")) is ws
