"""Two-stage Householder orthogonalization on AMD MI355X (gfx950).

Python binding of libtho (hand-written HIP kernels behind a C ABI, declared
in include/tho.h).  This layer only marshals arguments: it allocates outputs
and workspace with PyTorch on the tensors' device and calls the C entry
points on the current HIP stream.  Importing the package fails if libtho.so
has not been built.
"""

from . import _lib  # noqa: F401  (raises ImportError when libtho.so is absent)
from .api import (two_stage, two_stage_weighted, workspace_bytes, get_info, block_householder, BlockHouseholder, bcgs, hhqr_full, hhqr_full_workspace_bytes,  # noqa: F401
                  two_stage_backward, two_stage_autograd, TwoStageFunction,
                  BatchedPlan, two_stage_batched)

__all__ = ["two_stage", "two_stage_weighted", "workspace_bytes", "get_info", "block_householder", "BlockHouseholder", "bcgs", "hhqr_full", "hhqr_full_workspace_bytes", "two_stage_backward",
           "two_stage_autograd", "TwoStageFunction", "BatchedPlan", "two_stage_batched"]
