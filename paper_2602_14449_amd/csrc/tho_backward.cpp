// Reverse-mode adjoint of the map (V, A) -> (Q, R, S) computed by
// tho_two_stage (Algorithm 1, second choice of P), real FP64 (the complex128
// adjoint, the same steps with conjugate transposes, is in tho_complex.cpp).
//
// The paper does not treat differentiation; this is the exact adjoint of the
// forward steps, taken in reverse order:
//   (Q)     Q = [0; Q_] - W N, N = T^{-1} G, G = W^T [0; Q_]
//   (QR)    A1_low = Q_ R           (thin-QR adjoint, diag R > 0)
//   (S)     S = P^T A1_top
//   (A)     A1 = A - W Z, Z = T^{-T} W^T A
//   (W)     W = [P; 0] - V
//   (P, T)  V_top = Q1 R1, P = -Q1, T = I + R1^T   (square-QR adjoint)
// where the thin-QR adjoint of X = Q R is
//   X_bar = (Q_bar + Q copyltu(M)) R^{-T},  M = R R_bar^T - Q_bar^T Q.
// Nothing of the forward pass is stored beyond (Q, R): P and T come from the
// QR of V_top again, Z from the reduction W^T A, N from W^T Q = -T^T N (valid
// for orthonormal V, since W^T W = T + T^T), and Q_ = Q_low - V_low N.
// The n-sized work is four split-n reductions over rows of V (against A, Q,
// the Q adjoint and the A1 adjoint), one k x k reduction over the bottom
// rows, and row-streaming products for Q_, its adjoint and the outputs.
#include <algorithm>

#include "tho_host.h"

using namespace tho;

namespace {

struct BwdPlan {
    int KP, K0P, QP0;
    XtyPlan xp;
    double *part, *C3, *CA, *CQ, *CG, *CA1, *Z, *N, *Gb, *Yb;
    double *Qu, *Qub;
    double *MQ, *gRu, *Mk, *CL, *RT, *RiT, *CM;
    double *Pm, *Tm, *Tb, *A1t, *Pb, *TmI, *TbL, *M1, *CL1, *B1m, *Li;
    double* pk[4];
    size_t bytes;
};

void make_bwd_plan(int64_t n, int64_t k0, int64_t k, void* ws, BwdPlan& P) {
    Carve cv(ws);
    P.KP = kp_of(k);
    P.K0P = k0p_of(k0);
    P.QP0 = k0 > 0 ? rows_gemm_qp((int)k0) : 16;
    P.xp = xty_plan(n);
    const size_t nk = (size_t)std::max(P.K0P, 16) * P.KP;
    const size_t kk = (size_t)P.KP * P.KP;
    const size_t k00 = (size_t)std::max<int64_t>(k0, 1) * std::max<int64_t>(k0, 1);
    P.part = cv.take((size_t)P.xp.nblk * std::max(3 * nk, kk));
    P.MQ = cv.take(kk);
    P.gRu = cv.take(kk);
    P.Mk = cv.take(kk);
    P.CL = cv.take(kk);
    P.RT = cv.take(kk);
    P.RiT = cv.take(kk);
    P.CM = cv.take(kk);
    const size_t pkn = (size_t)std::max(std::max(P.K0P, P.KP), 16) * std::max(P.QP0, P.KP);
    for (auto& p : P.pk) p = cv.take(pkn);
    if (k0 > 0) {
        // V^T [A, Q, G_Q] side by side (ld 3 KP)
        P.C3 = cv.take(3 * nk);
        P.CA = P.C3;
        P.CQ = P.C3 + P.KP;
        P.CG = P.C3 + 2 * P.KP;
        P.CA1 = cv.take(nk);
        P.Z = cv.take(nk);
        P.N = cv.take(nk);
        P.Gb = cv.take(nk);
        P.Yb = cv.take(nk);
        P.A1t = cv.take(nk);
        P.Qu = cv.take((size_t)(n - k0) * k);
        P.Qub = cv.take((size_t)(n - k0) * k);
        for (double** p : {&P.Pm, &P.Tm, &P.Tb, &P.Pb, &P.TmI, &P.TbL, &P.M1, &P.CL1, &P.B1m, &P.Li}) *p = cv.take(k00);
    } else {
        P.C3 = P.CA = P.CQ = P.CG = P.CA1 = P.Z = P.N = P.Gb = P.Yb = P.A1t = P.Qu = P.Qub = nullptr;
        P.Pm = P.Tm = P.Tb = P.Pb = P.TmI = P.TbL = P.M1 = P.CL1 = P.B1m = P.Li = nullptr;
    }
    P.bytes = cv.bytes();
}

RowsGemm rows(int64_t nrows, const double* X, int64_t ldx, double* Out, int64_t ldo, int q) {
    RowsGemm g{};
    g.nrows = nrows;
    g.X = X;
    g.ldx = ldx;
    g.Out = Out;
    g.ldo = ldo;
    g.q = q;
    g.nterm = 0;
    return g;
}

void add_term(RowsGemm& g, const double* Y, int64_t ldy, int p, int kpad, const double* B) {
    g.t[g.nterm++] = {Y, ldy, p, kpad, B};
}

}  // namespace

extern "C" {

int tho_two_stage_backward_workspace(int32_t dtype, int64_t n, int64_t k0, int64_t k, const tho_opts_t* opts,
                                     size_t* bytes) {
    int rc = check_common(dtype, n, k0, k);
    if (rc) return rc;
    if (!bytes) return set_err(-6, "bytes must not be NULL");
    (void)opts;
    if (k == 0) { *bytes = 0; return 0; }
    if (dtype == THO_C128) {
        if (!zsupported(k0, k)) return set_err(THO_E_UNSUPPORTED, "complex128 supports k0 <= 64, k <= 32");
        *bytes = ztwo_stage_backward_bytes(n, k0, k);
        return 0;
    }
    BwdPlan P;
    make_bwd_plan(n, k0, k, nullptr, P);
    *bytes = P.bytes;
    return 0;
}

int tho_two_stage_backward(int32_t dtype, int64_t n, int64_t k0, int64_t k, const void* V_, int64_t ldv,
                           const void* A_, int64_t lda, const void* Q_, int64_t ldq, const void* R_, int64_t ldr,
                           const void* gQ_, int64_t ldgq, const void* gR_, int64_t ldgr, const void* gS_,
                           int64_t ldgs, void* dV_, int64_t lddv, void* dA_, int64_t ldda, const tho_opts_t* opts,
                           void* ws, size_t ws_bytes, void* stream) {
    int rc = check_common(dtype, n, k0, k);
    if (rc) return rc;
    const bool cplx = dtype == THO_C128;
    const int64_t esz = cplx ? 16 : 8;
    if (cplx && !zsupported(k0, k)) return set_err(THO_E_UNSUPPORTED, "complex128 supports k0 <= 64, k <= 32");
    if (opts && (opts->p_choice != THO_P_QR || opts->panel != THO_PANEL_F64 || opts->flags != 0))
        return set_err(THO_E_UNSUPPORTED, "the adjoint supports p_choice=THO_P_QR, panel=THO_PANEL_F64 only");
    if (k == 0) return 0;
    if ((rc = check_io(k0, k, V_, ldv, A_, lda, Q_, ldq, R_, ldr, R_, k))) return rc;
    if (!gQ_) return set_err(-13, "gQ is NULL");
    if (ldgq < k) return set_err(-14, "ldgq < k");
    if (!gR_) return set_err(-15, "gR is NULL");
    if (ldgr < k) return set_err(-16, "ldgr < k");
    if (gS_ && ldgs < k) return set_err(-18, "ldgs < k");
    if (k0 > 0 && !dV_) return set_err(-19, "dV is NULL");
    if (k0 > 0 && lddv < k0) return set_err(-20, "lddv < k0");
    if (!dA_) return set_err(-21, "dA is NULL");
    if (ldda < k) return set_err(-22, "ldda < k");
    for (const void* p : {V_, A_, Q_, R_, gQ_, gR_, gS_, (const void*)dV_, (const void*)dA_})
        if (p && ((uintptr_t)p & (esz - 1))) return set_err(-13, "matrices must be aligned to their element size");
    {
        // dV (arg 19) and dA (arg 21) must not share elements with an input or each other
        struct Blk { const void* p; int64_t r, c, ld; };
        const Blk in[] = {{V_, n, k0, ldv}, {A_, n, k, lda}, {Q_, n, k, ldq}, {R_, k, k, ldr},
                          {gQ_, n, k, ldgq}, {gR_, k, k, ldgr}, {gS_, k0, k, ldgs}};
        const Blk dv{dV_, n, k0, lddv}, da{dA_, n, k, ldda};
        for (const Blk& b : in) {
            if (blocks_overlap(dv.p, dv.r, dv.c, dv.ld, b.p, b.r, b.c, b.ld, esz))
                return set_err(-19, "dV overlaps an input");
            if (blocks_overlap(da.p, da.r, da.c, da.ld, b.p, b.r, b.c, b.ld, esz))
                return set_err(-21, "dA overlaps an input");
        }
        if (blocks_overlap(dv.p, dv.r, dv.c, dv.ld, da.p, da.r, da.c, da.ld, esz))
            return set_err(-21, "dA overlaps dV");
    }
    if (!ws) return set_err(-24, "workspace is NULL");
    if (cplx) {
        if (ws_bytes < ztwo_stage_backward_bytes(n, k0, k)) return set_err(THO_E_WORKSPACE, "workspace too small");
        return run_ztwo_stage_backward(n, k0, k, (const dcplx*)V_, ldv, (const dcplx*)A_, lda, (const dcplx*)Q_, ldq,
                                       (const dcplx*)R_, ldr, (const dcplx*)gQ_, ldgq, (const dcplx*)gR_, ldgr,
                                       (const dcplx*)gS_, ldgs, (dcplx*)dV_, lddv, (dcplx*)dA_, ldda, ws,
                                       (hipStream_t)stream);
    }
    BwdPlan P;
    make_bwd_plan(n, k0, k, nullptr, P);
    if (ws_bytes < P.bytes) return set_err(THO_E_WORKSPACE, "workspace too small");
    make_bwd_plan(n, k0, k, ws, P);

    hipStream_t st = (hipStream_t)stream;
    const double* V = (const double*)V_;
    const double* A = (const double*)A_;
    const double* Q = (const double*)Q_;
    const double* R = (const double*)R_;
    const double* gQ = (const double*)gQ_;
    const double* gR = (const double*)gR_;
    const double* gS = (const double*)gS_;
    double* dV = (double*)dV_;
    double* dA = (double*)dA_;
    const int KP = P.KP, K0P = P.K0P, QP0 = P.QP0, ik = (int)k, ik0 = (int)k0;
    const int64_t m = n - k0;

    const double *Qu = Q, *Qub = gQ;
    int64_t ldqu = ldq, ldqub = ldgq;
    if (k0 > 0) {
        // P and T again, then Z, N and the N adjoint from three
        // reductions over all rows:  C_X = V^T X for X = A, Q, gQ.
        // The QR of V_top runs on a side stream beside the reductions and is
        // joined before the first use of P and T.
        Fork& f = fork_for_thread();
        if (!f.ok) return set_err(THO_E_HIP, "could not create the side stream");
        HIPCHK(hipEventRecord(f.ev0, st));
        HIPCHK(hipStreamWaitEvent(f.side, f.ev0, 0));
        PROF("qr_top", f.side, launch_qr_top(ik0, V, ldv, P.Pm, P.Tm, f.side));
        HIPCHK(hipEventRecord(f.ev1, f.side));
        // the three reductions in one pass over V
        PROF("xty3_partial", st, launch_xty3_partial(K0P / 16, KP / 16, n, V, ldv, ik0, A, lda, Q, ldq, gQ, ldgq, ik,
                                                     P.xp.nblk, P.xp.rows_per_blk, P.part, st));
        PROF("reduce_parts", st, launch_reduce_parts(P.xp.nblk, (int64_t)K0P * 3 * KP, P.part, P.C3, st));
        HIPCHK(hipStreamWaitEvent(st, f.ev1, 0));
        // Z = T^{-T} W^T A,  W^T A = P^T A_top - V^T A
        PROF("small_gemm", st, launch_small_gemm(ik0, ik, ik0, 1.0, P.Pm, k0, 1, A, lda, 0, -1.0, P.CA, 3 * KP, P.Z, KP, st));
        PROF("trsm", st, launch_trsm_lower(ik0, ik, P.Tm, k0, 1, P.Z, KP, st));
        // N = -T^{-T} W^T Q
        PROF("small_gemm", st, launch_small_gemm(ik0, ik, ik0, -1.0, P.Pm, k0, 1, Q, ldq, 0, 1.0, P.CQ, 3 * KP, P.N, KP, st));
        PROF("trsm", st, launch_trsm_lower(ik0, ik, P.Tm, k0, 1, P.N, KP, st));
        // (Q) adjoint: N_bar = -W^T Q_bar, G_bar = T^{-T} N_bar
        PROF("small_gemm", st, launch_small_gemm(ik0, ik, ik0, -1.0, P.Pm, k0, 1, gQ, ldgq, 0, 1.0, P.CG, 3 * KP, P.Gb, KP,
                                                 st));
        PROF("trsm", st, launch_trsm_lower(ik0, ik, P.Tm, k0, 1, P.Gb, KP, st));
        // Q_ = Q_low - V_low N ;  Q__bar = Q_bar_low - V_low G_bar  (X_bar = Q_bar + W G_bar)
        PROF("pack_b", st, launch_pack_b(ik0, ik, P.N, KP, 0, -1.0, K0P, KP, P.pk[0], st));
        PROF("pack_b", st, launch_pack_b(ik0, ik, P.Gb, KP, 0, -1.0, K0P, KP, P.pk[1], st));
        RowsGemm g1 = rows(m, Q + k0 * ldq, ldq, P.Qu, k, ik);
        add_term(g1, V + k0 * ldv, ldv, ik0, K0P, P.pk[0]);
        PROF("rows_gemm", st, launch_rows_gemm(g1, st));
        RowsGemm g2 = rows(m, gQ + k0 * ldgq, ldgq, P.Qub, k, ik);
        add_term(g2, V + k0 * ldv, ldv, ik0, K0P, P.pk[1]);
        PROF("rows_gemm", st, launch_rows_gemm(g2, st));
        Qu = P.Qu;
        Qub = P.Qub;
        ldqu = ldqub = k;
    }

    // (QR) adjoint: A1_bar_low = Q__bar R^{-T} + Q_ (copyltu(M) R^{-T}),
    // M = R triu(R_bar)^T - Q__bar^T Q_
    if ((rc = xty(P.xp, m, Qub, ldqub, ik, Qu, ldqu, ik, P.part, P.MQ, st, "xty_qr_adj"))) return rc;
    PROF("small_ew", st, launch_small_ew(ik, ik, 1.0, gR, ldgr, 0, 0.0, nullptr, 0, 0, 0.0, 2, P.gRu, KP, st));
    PROF("small_gemm", st, launch_small_gemm(ik, ik, ik, 1.0, R, ldr, 0, P.gRu, KP, 1, -1.0, P.MQ, KP, P.Mk, KP, st));
    PROF("small_ew", st, launch_small_ew(ik, ik, 1.0, P.Mk, KP, 0, 0.0, nullptr, 0, 0, 0.0, 3, P.CL, KP, st));
    PROF("small_ew", st, launch_small_ew(ik, ik, 1.0, R, ldr, 1, 0.0, nullptr, 0, 0, 0.0, 1, P.RT, KP, st));
    PROF("small_ew", st, launch_small_ew(ik, ik, 0.0, nullptr, 0, 0, 0.0, nullptr, 0, 0, 1.0, 0, P.RiT, KP, st));
    PROF("trsm", st, launch_trsm_lower(ik, ik, P.RT, KP, 0, P.RiT, KP, st));
    PROF("small_gemm", st, launch_small_gemm(ik, ik, ik, 1.0, P.CL, KP, 0, P.RiT, KP, 0, 0.0, nullptr, 0, P.CM, KP, st));
    PROF("pack_b", st, launch_pack_b(ik, ik, P.RiT, KP, 0, 1.0, KP, KP, P.pk[2], st));
    PROF("pack_b", st, launch_pack_b(ik, ik, P.CM, KP, 0, 1.0, KP, KP, P.pk[3], st));
    {
        RowsGemm g = rows(m, nullptr, 0, dA + k0 * ldda, ldda, ik);
        add_term(g, Qub, ldqub, ik, KP, P.pk[2]);
        add_term(g, Qu, ldqu, ik, KP, P.pk[3]);
        PROF("rows_gemm", st, launch_rows_gemm(g, st));
    }
    if (k0 == 0) return 0;  // plain Householder QR: A_bar = A1_bar

    // (S) adjoint: A1_bar_top = P S_bar
    if (gS)
        PROF("small_gemm", st, launch_small_gemm(ik0, ik, ik0, 1.0, P.Pm, k0, 0, gS, ldgs, 0, 0.0, nullptr, 0, dA, ldda,
                                                 st));
    else
        PROF("small_ew", st, launch_small_ew(ik0, ik, 0.0, nullptr, 0, 0, 0.0, nullptr, 0, 0, 0.0, 0, dA, ldda, st));
    // (A) adjoint: Z_bar = -W^T A1_bar, Y_bar = T^{-1} Z_bar
    if ((rc = xty(P.xp, n, V, ldv, ik0, dA, ldda, ik, P.part, P.CA1, st, "xty_partial"))) return rc;
    PROF("small_gemm", st, launch_small_gemm(ik0, ik, ik0, -1.0, P.Pm, k0, 1, dA, ldda, 0, 1.0, P.CA1, KP, P.Yb, KP,
                                             st));
    PROF("trsm", st, launch_trsm_lower(ik0, ik, P.Tm, k0, 0, P.Yb, KP, st));
    // T_bar = -G_bar N^T - Z Y_bar^T
    PROF("small_gemm", st, launch_small_gemm(ik0, ik0, ik, -1.0, P.Gb, KP, 0, P.N, KP, 1, 0.0, nullptr, 0, P.Tb, k0,
                                             st));
    PROF("small_gemm", st, launch_small_gemm(ik0, ik0, ik, -1.0, P.Z, KP, 0, P.Yb, KP, 1, 1.0, P.Tb, k0, P.Tb, k0, st));
    // V_bar = -W_bar = Q_bar N^T - [0; Q_] G_bar^T + A1_bar Z^T - A Y_bar^T
    PROF("pack_b", st, launch_pack_b(ik, ik0, P.N, KP, 1, 1.0, KP, QP0, P.pk[0], st));
    PROF("pack_b", st, launch_pack_b(ik, ik0, P.Z, KP, 1, 1.0, KP, QP0, P.pk[1], st));
    PROF("pack_b", st, launch_pack_b(ik, ik0, P.Yb, KP, 1, -1.0, KP, QP0, P.pk[2], st));
    PROF("pack_b", st, launch_pack_b(ik, ik0, P.Gb, KP, 1, -1.0, KP, QP0, P.pk[3], st));
    // the top k0 rows take three terms, the bottom rows also - Q_ G_bar^T
    // (one pass over them)
    {
        RowsGemm g = rows(k0, nullptr, 0, dV, lddv, ik0);
        add_term(g, gQ, ldgq, ik, KP, P.pk[0]);
        add_term(g, dA, ldda, ik, KP, P.pk[1]);
        add_term(g, A, lda, ik, KP, P.pk[2]);
        PROF("rows_gemm", st, launch_rows_gemm(g, st));
    }
    {
        RowsGemm g = rows(m, nullptr, 0, dV + k0 * lddv, lddv, ik0);
        add_term(g, gQ + k0 * ldgq, ldgq, ik, KP, P.pk[0]);
        add_term(g, dA + k0 * ldda, ldda, ik, KP, P.pk[1]);
        add_term(g, A + k0 * lda, lda, ik, KP, P.pk[2]);
        add_term(g, P.Qu, k, ik, KP, P.pk[3]);
        PROF("rows_gemm", st, launch_rows_gemm(g, st));
    }
    // P_bar = A1_top S_bar^T + W_bar_top,  A1_top = A_top - (P - V_top) Z
    PROF("small_gemm", st, launch_small_gemm(ik0, ik, ik0, -1.0, P.Pm, k0, 0, P.Z, KP, 0, 1.0, A, lda, P.A1t, KP, st));
    PROF("small_gemm", st, launch_small_gemm(ik0, ik, ik0, 1.0, V, ldv, 0, P.Z, KP, 0, 1.0, P.A1t, KP, P.A1t, KP, st));
    if (gS)
        PROF("small_gemm", st, launch_small_gemm(ik0, ik0, ik, 1.0, P.A1t, KP, 0, gS, ldgs, 1, -1.0, dV, lddv, P.Pb, k0,
                                                 st));
    else
        PROF("small_ew", st, launch_small_ew(ik0, ik0, -1.0, dV, lddv, 0, 0.0, nullptr, 0, 0, 0.0, 0, P.Pb, k0, st));
    // A_bar = A1_bar + W Y_bar:  bottom rows - V_low Y_bar, top rows + (P - V_top) Y_bar
    PROF("pack_b", st, launch_pack_b(ik0, ik, P.Yb, KP, 0, -1.0, K0P, KP, P.pk[0], st));
    {
        RowsGemm g = rows(m, dA + k0 * ldda, ldda, dA + k0 * ldda, ldda, ik);
        add_term(g, V + k0 * ldv, ldv, ik0, K0P, P.pk[0]);
        PROF("rows_gemm", st, launch_rows_gemm(g, st));
    }
    PROF("small_gemm", st, launch_small_gemm(ik0, ik, ik0, 1.0, P.Pm, k0, 0, P.Yb, KP, 0, 1.0, dA, ldda, dA, ldda, st));
    PROF("small_gemm", st, launch_small_gemm(ik0, ik, ik0, -1.0, V, ldv, 0, P.Yb, KP, 0, 1.0, dA, ldda, dA, ldda, st));
    // (P, T) adjoint: square QR V_top = Q1 R1 with Q1 = -P, R1 = (T - I)^T,
    // Q1_bar = -P_bar, R1_bar = tril(T_bar)^T:
    //   M1 = R1 R1_bar^T - Q1_bar^T Q1 = (T - I)^T tril(T_bar) - P_bar^T P
    //   V_bar_top += (-P_bar - P copyltu(M1)) (T - I)^{-1}
    PROF("small_ew", st, launch_small_ew(ik0, ik0, 1.0, P.Tm, k0, 0, 0.0, nullptr, 0, 0, -1.0, 1, P.TmI, k0, st));
    PROF("small_ew", st, launch_small_ew(ik0, ik0, 1.0, P.Tb, k0, 0, 0.0, nullptr, 0, 0, 0.0, 1, P.TbL, k0, st));
    PROF("small_gemm", st, launch_small_gemm(ik0, ik0, ik0, 1.0, P.TmI, k0, 1, P.TbL, k0, 0, 0.0, nullptr, 0, P.M1, k0,
                                             st));
    PROF("small_gemm", st, launch_small_gemm(ik0, ik0, ik0, -1.0, P.Pb, k0, 1, P.Pm, k0, 0, 1.0, P.M1, k0, P.M1, k0,
                                             st));
    PROF("small_ew", st, launch_small_ew(ik0, ik0, 1.0, P.M1, k0, 0, 0.0, nullptr, 0, 0, 0.0, 3, P.CL1, k0, st));
    PROF("small_gemm", st, launch_small_gemm(ik0, ik0, ik0, -1.0, P.Pm, k0, 0, P.CL1, k0, 0, -1.0, P.Pb, k0, P.B1m, k0,
                                             st));
    PROF("small_ew", st, launch_small_ew(ik0, ik0, 0.0, nullptr, 0, 0, 0.0, nullptr, 0, 0, 1.0, 0, P.Li, k0, st));
    PROF("trsm", st, launch_trsm_lower(ik0, ik0, P.TmI, k0, 0, P.Li, k0, st));
    PROF("small_gemm", st, launch_small_gemm(ik0, ik0, ik0, 1.0, P.B1m, k0, 0, P.Li, k0, 0, 1.0, dV, lddv, dV, lddv,
                                             st));
    return 0;
}

}  // extern "C"
