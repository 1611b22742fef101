// Block classical Gram-Schmidt baseline (eq. (1) and the repetition
// patterns of Table 1): each round runs `proj` projections
//   C = V^T X,  X <- X - V C,  S_r += C          (BQR-1)
// and one Householder QR X = Q_r R_r (BQR-2, the chunked TSQR); the totals
// are S = S_1 + S_2 R_1 + S_3 R_2 R_1 + ... and R = R_r ... R_1.
// X lives in the caller's Q buffer from the first projection on.
#include <algorithm>

#include "tho_host.h"

using namespace tho;

namespace {

struct BcgsPlan {
    int KP, K0P;
    XtyPlan xp;
    TsqrPlan ts;
    double *part, *Cbuf, *Cpk, *Sr, *Rr, *Rtmp;
    size_t bytes;
};

void make_bcgs_plan(int64_t n, int64_t k0, int64_t k, void* ws, BcgsPlan& P) {
    Carve cv(ws);
    P.KP = kp_of(k);
    P.K0P = k0p_of(k0);
    P.xp = xty_plan(n);
    tsqr_plan(n, (int)k, cv, P.ts);
    const size_t nk = (size_t)std::max(P.K0P, 16) * P.KP;
    P.part = P.Cbuf = P.Cpk = P.Sr = nullptr;
    if (k0 > 0) {
        P.part = cv.take((size_t)P.xp.nblk * nk);
        P.Cbuf = cv.take(nk);
        P.Cpk = cv.take(nk);
        P.Sr = cv.take(nk);
    }
    P.Rr = cv.take((size_t)P.KP * P.KP);
    P.Rtmp = cv.take((size_t)P.KP * P.KP);
    P.bytes = cv.bytes();
}

int check_pr(int32_t proj, int32_t rounds, int iproj, int irounds) {
    if (proj < 1 || proj > 8) return set_err(-iproj, "proj must be in [1, 8]");
    if (rounds < 1 || rounds > 8) return set_err(-irounds, "rounds must be in [1, 8]");
    return 0;
}

}  // namespace

extern "C" {

int tho_bcgs_workspace(int32_t dtype, int64_t n, int64_t k0, int64_t k, int32_t proj, int32_t rounds,
                       const tho_opts_t* opts, size_t* bytes) {
    int rc = check_common(dtype, n, k0, k);
    if (rc) return rc;
    if ((rc = check_pr(proj, rounds, 5, 6))) return rc;
    if (!bytes) return set_err(-8, "bytes must not be NULL");
    (void)opts;
    if (k == 0) { *bytes = 0; return 0; }
    if (dtype == THO_C128) {
        if (!zsupported(k0, k)) return set_err(THO_E_UNSUPPORTED, "complex128 supports k0 <= 64, k <= 32");
        *bytes = zbcgs_bytes(n, k0, k);
        return 0;
    }
    BcgsPlan P;
    make_bcgs_plan(n, k0, k, nullptr, P);
    *bytes = P.bytes;
    return 0;
}

int tho_bcgs(int32_t dtype, int64_t n, int64_t k0, int64_t k, const void* V_, int64_t ldv, const void* A_,
             int64_t lda, void* Q_, int64_t ldq, void* R_, int64_t ldr, void* S_, int64_t lds, int32_t proj,
             int32_t rounds, const tho_opts_t* opts, void* ws, size_t ws_bytes, void* stream) {
    int rc = check_common(dtype, n, k0, k);
    if (rc) return rc;
    if (opts && (opts->panel != THO_PANEL_F64 || opts->flags != 0 || opts->p_choice != THO_P_QR))
        return set_err(THO_E_UNSUPPORTED, "tho_bcgs supports panel=THO_PANEL_F64 only");
    if ((rc = check_pr(proj, rounds, 15, 16))) return rc;
    if (dtype == THO_C128 && !zsupported(k0, k))
        return set_err(THO_E_UNSUPPORTED, "complex128 supports k0 <= 64, k <= 32");
    if (k == 0) return 0;
    if ((rc = check_io(k0, k, V_, ldv, A_, lda, Q_, ldq, R_, ldr, S_, lds))) return rc;
    if ((rc = check_alias(n, k0, k, dtype == THO_C128 ? 16 : 8, V_, ldv, A_, lda, Q_, ldq, R_, ldr, S_, lds)))
        return rc;
    if (!ws) return set_err(-18, "workspace is NULL");
    if (dtype == THO_C128) {
        if (ws_bytes < zbcgs_bytes(n, k0, k)) return set_err(THO_E_WORKSPACE, "workspace too small");
        return run_zbcgs(n, k0, k, (const dcplx*)V_, ldv, (const dcplx*)A_, lda, (dcplx*)Q_, ldq, (dcplx*)R_, ldr,
                         (dcplx*)S_, lds, proj, rounds, ws, (hipStream_t)stream);
    }
    BcgsPlan P;
    make_bcgs_plan(n, k0, k, nullptr, P);
    if (ws_bytes < P.bytes) return set_err(THO_E_WORKSPACE, "workspace too small");
    make_bcgs_plan(n, k0, k, ws, P);

    hipStream_t st = (hipStream_t)stream;
    const double* V = (const double*)V_;
    const double* A = (const double*)A_;
    double* Q = (double*)Q_;
    double* R = (double*)R_;
    double* S = (double*)S_;
    const int KP = P.KP, K0P = P.K0P, ik = (int)k, ik0 = (int)k0;

    const double* X = A;  // current block: A, then the Q buffer
    int64_t ldx = lda;
    for (int r = 0; r < rounds; r++) {
        if (k0 > 0) {
            for (int p = 0; p < proj; p++) {
                // (BQR-1): C = V^T X ; X <- X - V C ; S_r += C
                rc = xty(P.xp, n, V, ldv, ik0, X, ldx, ik, P.part, P.Cbuf, st, "xty_partial");
                if (rc) return rc;
                PROF("pack_b", st, launch_pack_b(ik0, ik, P.Cbuf, KP, 0, -1.0, K0P, KP, P.Cpk, st));
                RowsGemm g{};
                g.nrows = n;
                g.X = X;
                g.ldx = ldx;
                g.Out = Q;
                g.ldo = ldq;
                g.q = ik;
                g.nterm = 1;
                g.t[0] = {V, ldv, ik0, K0P, P.Cpk};
                PROF("rows_gemm", st, launch_rows_gemm(g, st));
                X = Q;
                ldx = ldq;
                if (p == 0)
                    PROF("small_ew", st, launch_small_ew(ik0, ik, 1.0, P.Cbuf, KP, 0, 0.0, nullptr, 0, 0, 0.0, 0, P.Sr,
                                                         KP, st));
                else
                    PROF("small_ew", st, launch_small_ew(ik0, ik, 1.0, P.Sr, KP, 0, 1.0, P.Cbuf, KP, 0, 0.0, 0, P.Sr,
                                                         KP, st));
            }
        }
        // (BQR-2): X = Q_r R_r
        std::vector<TsqrLevel> Ls = tsqr_levels(P.ts, X, ldx, Q, ldq);
        rc = tsqr_factor(P.ts, Ls, 0, P.Rr, KP, st);
        if (rc) return rc;
        rc = tsqr_form0(P.ts, Ls, 0, st);
        if (rc) return rc;
        X = Q;
        ldx = ldq;
        if (r == 0) {
            if (k0 > 0)
                PROF("small_ew", st, launch_small_ew(ik0, ik, 1.0, P.Sr, KP, 0, 0.0, nullptr, 0, 0, 0.0, 0, S, lds, st));
            PROF("small_ew", st, launch_small_ew(ik, ik, 1.0, P.Rr, KP, 0, 0.0, nullptr, 0, 0, 0.0, 0, R, ldr, st));
        } else {
            // S += S_r R_acc ; R_acc <- R_r R_acc
            if (k0 > 0)
                PROF("small_gemm", st, launch_small_gemm(ik0, ik, ik, 1.0, P.Sr, KP, 0, R, ldr, 0, 1.0, S, lds, S, lds,
                                                         st));
            PROF("small_gemm", st, launch_small_gemm(ik, ik, ik, 1.0, P.Rr, KP, 0, R, ldr, 0, 0.0, nullptr, 0, P.Rtmp,
                                                     KP, st));
            PROF("small_ew", st, launch_small_ew(ik, ik, 1.0, P.Rtmp, KP, 0, 0.0, nullptr, 0, 0, 0.0, 0, R, ldr, st));
        }
    }
    return 0;
}

}  // extern "C"
