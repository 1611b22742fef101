"""Pins for the oracle's Algorithm 1 (second choice of P) and its baselines.

Each test checks the oracle against something other than itself:
  * the worked example of eq. (2) and Example 1 (§6.1), with the closed form
    of (Q, R, S) worked by hand (tests/golden/example_eq2.json);
  * Table 1 for the BCGS baseline (tests/golden/table1_bcgs.json);
  * brute force: Householder QR of [V, A] on tiny inputs;
  * the identities of the second choice of P (§3.2);
  * Theorem 1 on a densely formed H (§4);
  * special cases that reduce to a plain QR (k0 = 0, V_low = 0, A = 0);
  * the rounding bounds of Theorem 3 and its remarks (loss, ||V^*Q|| and
    residual independent of cond([V, A])), and the remark after Theorem 1
    (loss tracks ||V^*V - I|| for non-orthonormal V);
  * the second-choice row of Table 4 as an order-of-magnitude bound.
"""

import json
import os

import numpy as np
import pytest

import tho_workloads as W
from oracle import (two_stage, two_stage_intermediates, hhqr_full, bcgs,
                    qr_pos, orth_loss, orth_parts, rel_residual)

GOLD = os.path.join(os.path.dirname(__file__), "golden")
U = 2.0 ** -53


def _load(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def _phase_align(Q, Qref):
    """Scale columns of Q by unit phases to best match Qref."""
    d = np.sum(np.conj(Q) * Qref, axis=0)
    ph = np.where(np.abs(d) > 0, d / np.where(np.abs(d) > 0, np.abs(d), 1), 1)
    return Q * ph[None, :]


# ---------------------------------------------------------------- eq. (2)

def test_worked_example_closed_form():
    gold = _load("example_eq2.json")
    V, A = W.example2()
    assert np.allclose(V, np.array(gold["V"]), atol=0, rtol=1e-16)
    assert np.array_equal(A, np.array(gold["A"]))
    o = two_stage_intermediates(V, A)
    # second choice on this V: R1 = I, P = -V_top, T = 2I
    assert np.allclose(o["R1"], np.eye(2), atol=4 * U)
    assert np.allclose(o["P"], -V[:2], atol=4 * U)
    assert np.allclose(o["T"], 2 * np.eye(2), atol=4 * U)
    Q, R, S = o["Q"], o["R"], o["S"]
    assert np.allclose(Q, np.array(gold["Q"]), atol=1e-15)
    assert np.allclose(R, np.array(gold["R"]), rtol=1e-14, atol=1e-45)
    assert np.allclose(S, np.array(gold["S"]), atol=1e-15)
    loss = orth_loss(V, Q)
    # Example 1: ~2u; allow a small multiple of u
    assert loss <= 4 * gold["printed_loss_approx"]
    assert rel_residual(V, A, Q, R, S) < 1e-15


def test_worked_example_bcgs_fails_twostage_succeeds():
    V, A = W.example2()
    Qb, Rb, Sb = bcgs(V, A, proj=1, rounds=1)
    Qt, Rt, St = two_stage(V, A)
    assert orth_loss(V, Qb) > 0.5
    assert orth_loss(V, Qt) < 1e-15


def test_table1_bcgs_patterns():
    gold = _load("table1_bcgs.json")
    V, A = W.example2()
    for row in gold["rows"]:
        Q, R, S = bcgs(V, A, proj=row["proj"], rounds=row["rounds"])
        loss = orth_loss(V, Q)
        p = row["printed"]
        if p >= 0.5:
            assert loss >= 0.5, row
        elif p > 1e-10:
            assert p / 2 <= loss <= p * 2, (row, loss)
        else:
            assert loss <= 5 * p, (row, loss)
        # BCGS still reproduces A (eq. (1) keeps the residual small)
        assert rel_residual(V, A, Q, R, S) < 1e-14


# ---------------------------------------------------------- brute force

@pytest.mark.parametrize("seed", range(12))
def test_brute_force_against_full_householder(seed):
    g = np.random.default_rng(100 + seed)
    cplx = seed % 3 == 2
    n = int(g.integers(6, 64))
    k0 = int(g.integers(1, max(2, n // 3)))
    k = int(g.integers(1, max(2, n - k0 - 1)))
    k = min(k, n - k0)
    Vg = g.standard_normal((n, k0)) + (1j * g.standard_normal((n, k0)) if cplx else 0)
    V, _ = np.linalg.qr(Vg)
    A = g.standard_normal((n, k)) + (1j * g.standard_normal((n, k)) if cplx else 0)
    Qt, Rt, St = two_stage(V, A)
    Qh, Rh, Sh = hhqr_full(V, A)
    assert np.allclose(Qt, Qh, atol=1e-11)
    assert np.allclose(Rt, Rh, atol=1e-11)
    assert np.allclose(St, Sh, atol=1e-11)
    assert np.allclose(St, np.conj(V).T @ A, atol=1e-12)


def test_n_equals_k0_plus_k():
    g = np.random.default_rng(5)
    V, _ = np.linalg.qr(g.standard_normal((12, 7)))
    A = g.standard_normal((12, 5))
    Qt, Rt, St = two_stage(V, A)
    assert orth_loss(V, Qt) < 1e-14
    assert rel_residual(V, A, Qt, Rt, St) < 1e-14


# ------------------------------------------------- choice-2 identities

@pytest.mark.parametrize("cplx", [False, True])
def test_second_choice_identities(cplx):
    g = np.random.default_rng(21)
    n, k0, k = 4096, 16, 8
    V = W.orthonormal(g, n, k0, complex_=cplx)
    A = W.gaussian(g, (n, k), complex_=cplx)
    o = two_stage_intermediates(V, A)
    T, Wm, P = o["T"], o["W"], o["P"]
    assert np.allclose(np.triu(T, 1), 0)                      # lower triangular
    assert np.all(np.real(np.diag(T)) >= 1 - 1e-15)
    assert np.allclose(np.imag(np.diag(T)), 0)
    assert np.linalg.norm(T, 2) <= 2 + 1e-14                  # ||T||_2 <= 2
    WW = np.conj(Wm).T @ Wm
    assert np.allclose(T + np.conj(T).T, WW, atol=1e-13)      # T + T^* = W^*W
    assert np.allclose(np.sum(np.abs(Wm) ** 2, axis=0), 2 * np.real(np.diag(T)),
                       atol=1e-13)                            # ||w_i||^2 = 2 T_ii
    Ti = np.linalg.inv(T)
    assert np.max(np.abs(Ti)) <= 2 + 1e-12                    # |(T^-1)_ij| <= 2
    assert np.linalg.cond(T) < 2 * np.sqrt(2) * k0            # kappa(T) < 2 sqrt2 k0
    # T as written in Algorithm 1 versus the Appendix B.2 form
    T_line3 = np.eye(k0) - np.conj(V[:k0]).T @ P
    assert np.linalg.norm(T - T_line3, 2) < 1e-14


def test_theorem1_dense_H():
    g = np.random.default_rng(2)
    n, k0, k = 40, 6, 4
    V = W.orthonormal(g, n, k0)
    A = g.standard_normal((n, k))
    o = two_stage_intermediates(V, A)
    Wm, T, P = o["W"], o["T"], o["P"]
    H = np.eye(n) - Wm @ np.linalg.solve(T, Wm.T)
    X = np.zeros((n, k0))
    X[:k0] = P
    assert np.linalg.norm(H @ X - V, 2) < 1e-14               # H X = Y
    assert np.linalg.norm(H.T @ H - np.eye(n), 2) < 1e-14     # unitary
    assert np.linalg.norm(H.T @ V - X, 2) < 1e-14             # H^* Y = X
    # the update of A equals H^* A, the formation of Q equals H [0; Q_]
    assert np.allclose(o["A1"], H.T @ A, atol=1e-13)
    Xq = np.zeros((n, k))
    Xq[k0:] = o["Qu"]
    assert np.allclose(o["Q"], H @ Xq, atol=1e-14)


# ------------------------------------------------------- special cases

def test_k0_zero_is_plain_qr():
    g = np.random.default_rng(4)
    A = g.standard_normal((50, 6))
    Q, R, S = two_stage(np.zeros((50, 0)), A)
    Qr, Rr = qr_pos(A)
    assert np.allclose(Q, Qr) and np.allclose(R, Rr) and S.shape == (0, 6)


def test_v_low_zero():
    # V = [U; 0]: W_low = 0, so Q = [0; qr(A_low)] and S = U^T A_top
    g = np.random.default_rng(8)
    n, k0, k = 30, 5, 4
    Uo, _ = np.linalg.qr(g.standard_normal((k0, k0)))
    V = np.zeros((n, k0))
    V[:k0] = Uo
    A = g.standard_normal((n, k))
    Q, R, S = two_stage(V, A)
    Qr, Rr = qr_pos(A[k0:])
    assert np.allclose(Q[:k0], 0, atol=1e-15)
    assert np.allclose(Q[k0:], Qr, atol=1e-14)
    assert np.allclose(R, Rr, atol=1e-14)
    assert np.allclose(S, Uo.T @ A[:k0], atol=1e-14)


def test_a_zero_and_a_in_range_v():
    g = np.random.default_rng(9)
    n, k0, k = 200, 10, 5
    V = W.orthonormal(g, n, k0)
    for A in (np.zeros((n, k)), V @ g.standard_normal((k0, k))):
        Q, R, S = two_stage(V, A)
        assert orth_loss(V, Q) < 1e-14
        assert np.linalg.norm(A - V @ S - Q @ R, 2) < 1e-13 * max(1, np.linalg.norm(A, 2))
        assert np.linalg.norm(R, 2) < 1e-13 * max(1, np.linalg.norm(A, 2))


# ----------------------------------------------- Theorem 3 and remarks

@pytest.mark.parametrize("cond", [1e2, 1e8, 1e12, 1e16])
def test_stability_independent_of_conditioning(cond):
    V, A = W.graded(n=4096, k0=32, k=16, cond=cond, seed_cfg=30)
    Q, R, S = two_stage(V, A)
    assert orth_loss(V, Q) < 1e-13
    vq, qq = orth_parts(V, Q)
    assert vq < 1e-14 and qq < 1e-13
    assert rel_residual(V, A, Q, R, S) < 1e-14


def test_bcgs_breaks_on_ill_conditioned_complex_case():
    # the complex workload's structure at a smaller n: [V, A] has condition ~1e10
    V, A = W.complex_case(n=1 << 13, k0=16, k=8, seed_cfg=31)
    Qb, _, _ = bcgs(V, A, proj=1, rounds=1)
    Qt, Rt, St = two_stage(V, A)
    assert orth_loss(V, Qb) > 1e-9
    assert orth_loss(V, Qt) < 1e-13
    assert rel_residual(V, A, Qt, Rt, St) < 1e-14


def test_non_orthonormal_v_loss_tracks_delta():
    g = np.random.default_rng(12)
    n, k0, k = 2000, 8, 4
    V0 = W.orthonormal(g, n, k0)
    A = g.standard_normal((n, k))
    losses, deltas = [], []
    for delta in (1e-10, 1e-8, 1e-6):
        V = V0 @ (np.eye(k0) + delta * np.diag(np.linspace(-1, 1, k0)))
        d1 = np.linalg.norm(V.T @ V - np.eye(k0), 2)
        Q, R, S = two_stage(V, A)
        vq, qq = orth_parts(V, Q)
        losses.append(qq + vq)
        deltas.append(d1)
    # linear in delta_1 = ||V^T V - I||_2 (Theorem 1 bound, remark after it)
    for lo, d1 in zip(losses, deltas):
        assert 1e-3 * d1 < lo < 10 * d1
    assert 50 < losses[1] / losses[0] < 200 and 50 < losses[2] / losses[1] < 200


def test_table4_second_choice_order_of_magnitude():
    gold = _load("table4_badmlu.json")["rows"]["second choice"]
    g = np.random.default_rng(44)
    V = W.orthonormal(g, 1000, 100)
    A = g.standard_normal((1000, 100))
    Q, R, S = two_stage(V, A)
    vq, qq = orth_parts(V, Q)
    res = rel_residual(V, A, Q, R, S)
    assert vq < 10 * gold[0] and qq < 10 * gold[1] and res < 10 * gold[2]


def test_two_stage_vs_full_hhqr_plain_workload():
    V, A = W.plain()
    Qt, Rt, St = two_stage(V, A)
    Qh, Rh, Sh = hhqr_full(V, A)
    assert orth_loss(V, Qt) < 1e-14 and orth_loss(V, Qh) < 1e-14
    assert np.max(np.abs(_phase_align(Qt, Qh) - Qh)) < 1e-12
    assert np.allclose(Rt, Rh, atol=1e-12) and np.allclose(St, Sh, atol=1e-12)


def test_bcgs_reorth_agrees_on_well_conditioned():
    V, A = W.plain(n=1024, k0=8, k=4, seed_cfg=40)
    Qb, Rb, Sb = bcgs(V, A, proj=2, rounds=1)
    Qt, Rt, St = two_stage(V, A)
    assert np.allclose(Qb, Qt, atol=1e-12)
    assert np.allclose(Rb, Rt, atol=1e-12)
    assert np.allclose(Sb, St, atol=1e-12)
