"""Plain FP64 CPU oracle for two-stage Householder orthogonalization.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) may import, call or link anything here.  The only permitted
users are ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg
of ``bench.py``.

The oracle is written from He & Shao, "On Two-Stage Householder
Orthogonalization" (arXiv 2602.14449).  Every function cites the passage it
follows (section, equation, algorithm or table).  All arithmetic is IEEE
double (real float64 or complex128), the precision the paper's experiments
use (start of §6).  Library primitives (matrix products, triangular solves,
LAPACK QR for very tall inputs, eigenvalues for 2-norms) are used as single
steps; nothing is blocked, fused or reordered beyond what the paper states.

Modules
  householder  column Householder QR (the intra-block QR of
               Algorithm 1 and the QR of the top block for the second choice
               of P), with the nonnegative-diagonal phase convention
  choices      the three choices of P and the factored T they give (§3.2:
               modified LU of Algorithm 2, QR, polar decomposition)
  two_stage    the two-stage method from the definitions of §3.1 (eq. (3),
               eq. (4)), any choice of P
  b_inner      the two-stage method in a B-inner product (Algorithm 3,
               Theorem 4, §5) and its definition through the Cholesky
               transform
  block_householder  Algorithm 4 (block Householder-QR, §6.1) and the block
               BCGS2 baseline of Table 5
  appendix_a   the matrix U of eq. (6) and the Appendix A construction of an
               orthonormal V whose modified LU returns it (Example 4)
  baselines    Householder QR of [V, A] (start of §3) and the BCGS framework
               with reorthogonalization patterns (eq. (1), Table 1)
  metrics      loss of orthogonality and residual as printed in Tables 1-4
  adjoint      reverse-mode gradient of the map Algorithm 1 computes, plus a
               central finite-difference checker (the paper is silent on
               gradients; see the module header)

Parity status: every function here is pinned by ``tests/test_oracle_*.py``;
the reduced-precision panel variants of the GPU library have no oracle of
their own ("parity unpinned": their loss is reported against this FP64
oracle).
"""

from .householder import householder_qr, qr_pos, phase_normalize  # noqa: F401
from .two_stage import two_stage, two_stage_intermediates  # noqa: F401
from .choices import choose_p, modified_lu, polar  # noqa: F401
from .appendix_a import badmlu_u, badmlu_v  # noqa: F401
from .baselines import hhqr_full, bcgs  # noqa: F401
from .metrics import (  # noqa: F401
    orth_loss, orth_parts, rel_residual, gram_chunked, spectral_norm_tall)
