"""Pins for the three choices of P (§3.2, Algorithm 2, eq. (6), Appendix A,
Table 4) in the oracle.

Each test checks the oracle against something other than itself:
  * modified LU: the factorization P - Z = L U it defines, the pivot bound
    |U_ii| >= 1 stated with Algorithm 2, and the link to Householder QR of an
    orthonormal V ([BDGJKN2015, Lemma 6.2], used in Appendix A): its P equals
    the signs of diag(R) of LAPACK's Householder QR of V (library routine);
  * eq. (6): kappa_2(U) ~ 1.1e7 at k0 = 100, alpha = 0.1, as printed;
  * Appendix A: the constructed V is orthonormal and modified LU of its top
    block returns the U of eq. (6);
  * polar decomposition: scipy.linalg.polar (library routine), and the
    bound kappa_2(I + M) <= 2 of the third choice;
  * eq. (3): every factored T equals W^* X = I - V_top^* P;
  * exact arithmetic gives the same (Q, R, S) for every unitary P
    (Q = (I - V V^*) A R^{-1}), so the three choices agree with each other
    and with the Householder QR of [V, A] on well-conditioned inputs;
  * Theorem 1 on a densely formed H for every choice;
  * Table 4: all three rows.
"""

import json
import os

import numpy as np
import pytest
import scipy.linalg

import tho_workloads as W
from oracle import hhqr_full, orth_parts, rel_residual, two_stage, two_stage_intermediates
from oracle.appendix_a import badmlu_u, badmlu_v
from oracle.choices import choose_p, modified_lu, polar

GOLD = os.path.join(os.path.dirname(__file__), "golden")
CHOICES = ["mlu", "qr", "polar"]


def _table4():
    with open(os.path.join(GOLD, "table4_badmlu.json")) as f:
        return json.load(f)


@pytest.mark.parametrize("cplx", [False, True])
def test_modified_lu_factorization(cplx):
    g = np.random.default_rng(31)
    V = W.orthonormal(g, 200, 12, complex_=cplx)
    Z = V[:12]
    P, L, U = modified_lu(Z)
    assert np.allclose(P, np.diag(np.diag(P)))
    assert set(np.real(np.diag(P)).round().astype(int)) <= {-1, 1}
    assert np.allclose(np.imag(np.diag(P)), 0)
    assert np.allclose(np.triu(L, 1), 0) and np.allclose(np.diag(L), 1)
    assert np.allclose(np.tril(U, -1), 0)
    assert np.min(np.abs(np.diag(U))) >= 1.0 - 1e-15          # no pivoting needed
    assert np.linalg.norm(L @ U - (P - Z), 2) < 1e-14


def test_modified_lu_signs_follow_householder_qr():
    # Lemma 6.2 of [BDGJKN2015] (Appendix A): on an orthonormal V the Schur
    # complements of modified LU are the trailing matrices of Householder QR,
    # so P_ii = -sign(pivot) = the i-th diagonal entry of R from LAPACK's
    # Householder QR of V (beta = -sign(alpha) ||x||)
    for seed in range(3):
        g = np.random.default_rng(40 + seed)
        V = W.orthonormal(g, 300, 20)
        P, _, _ = modified_lu(V[:20])
        Rl = np.linalg.qr(V, mode="r")
        assert np.allclose(np.abs(np.diag(Rl)), 1, atol=1e-13)
        assert np.array_equal(np.diag(P), np.sign(np.diag(Rl)))


def test_eq6_condition_number():
    gold = _table4()["eq6"]
    U = badmlu_u(gold["k0"], gold["alpha"])
    kappa = np.linalg.cond(U)
    # printed to two digits: ~1.1e7
    assert 1.05e7 <= kappa < 1.15e7, kappa
    assert abs(kappa - gold["kappa2_U_approx"]) / gold["kappa2_U_approx"] < 0.05


def test_appendix_a_construction_yields_eq6():
    U = badmlu_u(100, 0.1)
    g = np.random.default_rng(7)
    V = badmlu_v(1000, U, g)
    assert V.shape == (1000, 100)
    assert np.linalg.norm(V.T @ V - np.eye(100), 2) < 1e-13
    P, L, Uc = modified_lu(V[:100])
    assert np.array_equal(np.diag(P), np.ones(100))
    # modified LU is forward-unstable exactly here (kappa(U) ~ 1e7): U is
    # reproduced to about kappa(U) u k0
    assert np.max(np.abs(Uc - U)) < 1e-5
    assert np.max(np.abs(Uc - U)) / np.max(np.abs(U)) < 1e-5
    # a small case is exact to rounding
    Us = badmlu_u(6, 0.1)
    Vs = badmlu_v(40, Us, np.random.default_rng(8))
    assert np.max(np.abs(modified_lu(Vs[:6])[2] - Us)) < 1e-14


@pytest.mark.parametrize("cplx", [False, True])
def test_polar_third_choice(cplx):
    g = np.random.default_rng(33)
    V = W.orthonormal(g, 64, 10, complex_=cplx)
    Vt = V[:10]
    Q2, M = polar(Vt)
    Q2s, Ms = scipy.linalg.polar(Vt, side="right")
    assert np.allclose(Q2, Q2s, atol=1e-12) and np.allclose(M, Ms, atol=1e-12)
    assert np.linalg.norm(np.conj(Q2).T @ Q2 - np.eye(10), 2) < 1e-14
    assert np.allclose(M, np.conj(M).T, atol=0)
    assert np.min(np.linalg.eigvalsh(M)) > -1e-14
    assert np.linalg.norm(Q2 @ M - Vt, 2) < 1e-14
    P, Tf = choose_p(Vt, "polar")
    assert np.linalg.cond(Tf.T) <= 2 + 1e-12                 # kappa_2(I + M) <= 2
    # a singular top block still gives a unitary P
    Vz = V.copy()
    Vz[:10, 3] = 0.0
    Q2z, Mz = polar(Vz[:10])
    assert np.linalg.norm(np.conj(Q2z).T @ Q2z - np.eye(10), 2) < 1e-14


@pytest.mark.parametrize("choice", CHOICES)
@pytest.mark.parametrize("cplx", [False, True])
def test_factored_t_matches_eq3(choice, cplx):
    g = np.random.default_rng(34)
    V = W.orthonormal(g, 500, 16, complex_=cplx)
    P, Tf = choose_p(V[:16], choice)
    assert np.linalg.norm(np.conj(P).T @ P - np.eye(16), 2) < 1e-14
    T3 = np.eye(16) - np.conj(V[:16]).T @ P          # T = W^* X
    assert np.linalg.norm(Tf.T - T3, 2) < 1e-13
    B = W.gaussian(g, (16, 5), complex_=cplx)
    assert np.allclose(T3 @ Tf.solve(B), B, atol=1e-12)
    assert np.allclose(np.conj(T3).T @ Tf.solve_h(B), B, atol=1e-12)


@pytest.mark.parametrize("cplx", [False, True])
def test_choices_agree_and_match_full_hhqr(cplx):
    g = np.random.default_rng(35)
    n, k0, k = 700, 24, 10
    V = W.orthonormal(g, n, k0, complex_=cplx)
    A = W.gaussian(g, (n, k), complex_=cplx)
    Qh, Rh, Sh = hhqr_full(V, A)
    for ch in CHOICES:
        Q, R, S = two_stage(V, A, p_choice=ch)
        assert np.max(np.abs(Q - Qh)) < 1e-12, ch
        assert np.max(np.abs(R - Rh)) < 1e-12, ch
        assert np.max(np.abs(S - Sh)) < 1e-12, ch


@pytest.mark.parametrize("choice", CHOICES)
def test_theorem1_dense_h_every_choice(choice):
    g = np.random.default_rng(36)
    n, k0, k = 40, 6, 4
    V = W.orthonormal(g, n, k0)
    A = g.standard_normal((n, k))
    o = two_stage_intermediates(V, A, p_choice=choice)
    Wm, T, P = o["W"], o["T"], o["P"]
    H = np.eye(n) - Wm @ np.linalg.solve(T, Wm.T)
    X = np.zeros((n, k0))
    X[:k0] = P
    assert np.linalg.norm(H @ X - V, 2) < 1e-14
    assert np.linalg.norm(H.T @ H - np.eye(n), 2) < 1e-14
    assert np.allclose(o["A1"], H.T @ A, atol=1e-13)
    Xq = np.zeros((n, k))
    Xq[k0:] = o["Qu"]
    assert np.allclose(o["Q"], H @ Xq, atol=1e-14)


def test_table4_all_rows():
    rows = _table4()["rows"]
    g = np.random.default_rng(7)
    V = badmlu_v(1000, badmlu_u(100, 0.1), g)
    A = g.standard_normal((1000, 100))
    got = {}
    for ch, name in zip(CHOICES, ["first choice", "second choice", "third choice"]):
        Q, R, S = two_stage(V, A, p_choice=ch)
        vq, qq = orth_parts(V, Q)
        got[name] = [vq, qq, rel_residual(V, A, Q, R, S)]
        print(name, "printed", rows[name], "oracle", ["%.2e" % x for x in got[name]])
    for name in ["second choice", "third choice"]:
        assert all(x < 10 * p for x, p in zip(got[name], rows[name])), name
    # the first choice loses accuracy through kappa(U): each quantity within
    # a factor of 10 of the printed value, and far above the stable choices
    for x, p, s in zip(got["first choice"], rows["first choice"], got["second choice"]):
        assert p / 10 < x < 10 * p
        assert x > 1e4 * s
