// C ABI of libtho: argument validation, workspace layout and the launch
// sequence of the two-stage Householder orthogonalization (Algorithm 1 of
// He & Shao, second choice of P) on one HIP stream.  No host
// synchronization and no device allocation happen here.
#include <algorithm>

#include "tho_host.h"

using namespace tho;

namespace {

struct TwoStagePlan {
    int KP, K0P;
    XtyPlan xp;
    TsqrPlan ts;
    double *part, *Cbuf, *Pm, *Tm, *Zbuf, *A1top, *Mbuf, *Nglob, *Nc, *prod, *Zperm, *Nperm;
    double *Zlp, *Nlp;  // reduced-precision panels only
    size_t bytes;
};

void make_plan(int64_t n, int64_t k0, int64_t k, void* ws, TwoStagePlan& P, int panel = 0) {
    Carve cv(ws);
    P.KP = kp_of(k);
    P.K0P = k0p_of(k0);
    P.xp = xty_plan(n);
    tsqr_plan(n - k0, (int)k, cv, P.ts);
    const size_t nk = (size_t)std::max(P.K0P, 16) * P.KP;
    const int nc0 = P.ts.lv[0].nchunk;
    if (k0 > 0) {
        P.part = cv.take((size_t)std::max(P.xp.nblk, nc0) * nk);
        P.Cbuf = cv.take(nk);
        P.Pm = cv.take((size_t)k0 * k0);
        P.Tm = cv.take((size_t)k0 * k0);
        P.Zbuf = cv.take(nk);
        P.A1top = cv.take((size_t)k0 * P.KP);
        P.Mbuf = cv.take(nk);
        P.Nglob = cv.take(nk);
        P.Nc = cv.take((size_t)nc0 * nk);
        P.Zperm = cv.take(nk);
        P.Nperm = cv.take(nk);
        P.prod = P.part;
        P.Zlp = P.Nlp = nullptr;
        if (panel != 0) {
            const size_t lb = lowp_pack_bytes(panel, P.K0P, P.KP) / sizeof(double) + 1;
            P.Zlp = cv.take(lb);
            P.Nlp = cv.take(lb);
        }
    } else {
        P.part = P.Cbuf = P.Pm = P.Tm = P.Zbuf = P.A1top = P.Mbuf = P.Nglob = P.Nc = P.prod = nullptr;
        P.Zperm = P.Nperm = P.Zlp = P.Nlp = nullptr;
    }
    P.bytes = cv.bytes();
}

}  // namespace

namespace tho {
int check_common(int32_t dtype, int64_t n, int64_t k0, int64_t k) {
    if (dtype != THO_F64 && dtype != THO_C128) return set_err(-1, "dtype must be THO_F64 or THO_C128");
    if (n < 0) return set_err(-2, "n must be >= 0");
    if (k0 < 0 || k0 > THO_MAX_K0) return set_err(-3, "k0 out of range [0, THO_MAX_K0]");
    if (k < 0 || k > THO_MAX_K) return set_err(-4, "k out of range [0, THO_MAX_K]");
    if (n < k0 + k) return set_err(-2, "need n >= k0 + k");
    return 0;
}

int check_io(int64_t k0, int64_t k, const void* V, int64_t ldv, const void* A, int64_t lda, const void* Q,
             int64_t ldq, const void* R, int64_t ldr, const void* S, int64_t lds) {
    if (k0 > 0 && !V) return set_err(-5, "V is NULL");
    if (k0 > 0 && ldv < k0) return set_err(-6, "ldv < k0");
    if (!A) return set_err(-7, "A is NULL");
    if (lda < k) return set_err(-8, "lda < k");
    if (!Q) return set_err(-9, "Q is NULL");
    if (ldq < k) return set_err(-10, "ldq < k");
    if (!R) return set_err(-11, "R is NULL");
    if (ldr < k) return set_err(-12, "ldr < k");
    if (k0 > 0 && !S) return set_err(-13, "S is NULL");
    if (k0 > 0 && lds < k) return set_err(-14, "lds < k");
    for (const void* p : {V, A, Q, R, S})
        if (p && ((uintptr_t)p & 7)) return set_err(-5, "matrices must be 8-byte aligned");
    return 0;
}
}  // namespace tho

namespace {

// Launch sequence of Algorithm 1 (second choice of P) on validated
// arguments; ws holds at least two_stage_bytes(n, k0, k).
int run_two_stage(int64_t n, int64_t k0, int64_t k, const double* V, int64_t ldv, const double* A, int64_t lda,
                  double* Q, int64_t ldq, double* R, int64_t ldr, double* S, int64_t lds, void* ws,
                  hipStream_t st, int panel = 0) {
    int rc = 0;
    if (k0 == 0) panel = 0;
    TwoStagePlan P;
    make_plan(n, k0, k, ws, P, panel);
    const int KP = P.KP, K0P = P.K0P;
    const int ik = (int)k, ik0 = (int)k0;
    const size_t nk = (size_t)std::max(K0P, 16) * KP;

    if (k0 > 0) {
        // P and T, second choice (§3.2): V_top = Q1 R1, P = -Q1, T = I + R1^T,
        // on a side stream, concurrently with the reduction C = V^T A over
        // all n rows (update of A); joined before the first use of P and T
        Fork& f = fork_for_thread();
        if (!f.ok) return set_err(THO_E_HIP, "could not create the side stream");
        HIPCHK(hipEventRecord(f.ev0, st));
        HIPCHK(hipStreamWaitEvent(f.side, f.ev0, 0));
        PROF("qr_top", f.side, launch_qr_top(ik0, V, ldv, P.Pm, P.Tm, f.side));
        HIPCHK(hipEventRecord(f.ev1, f.side));
        rc = xty(P.xp, n, V, ldv, ik0, A, lda, ik, P.part, P.Cbuf, st, "xty_partial", panel);
        if (rc) return rc;
        HIPCHK(hipStreamWaitEvent(st, f.ev1, 0));
        // W^T A = P^T A_top - C ;  Z = T^{-T} (W^T A)
        PROF("fill", st, fill(P.Zbuf, (int64_t)nk, 0.0, st));
        PROF("small_gemm", st, launch_small_gemm(ik0, ik, ik0, 1.0, P.Pm, k0, 1, A, lda, 0, -1.0, P.Cbuf, KP, P.Zbuf,
                                 KP, st));
        PROF("trsm", st, launch_trsm_lower(ik0, ik, P.Tm, k0, 1, P.Zbuf, KP, st));
        PROF("permute", st, launch_permute_b(K0P, KP, P.Zbuf, P.Zperm, st));
        if (panel) PROF("pack_lowp", st, launch_pack_b_lowp(panel, K0P, KP, P.Zbuf, P.Zlp, st));
        // A1_top = A_top - (P - V_top) Z ;  S = P^T A1_top
        PROF("small_gemm", st, launch_small_gemm(ik0, ik, ik0, -1.0, P.Pm, k0, 0, P.Zbuf, KP, 0, 1.0, A, lda, P.A1top,
                                 KP, st));
        PROF("small_gemm", st, launch_small_gemm(ik0, ik, ik0, 1.0, V, ldv, 0, P.Zbuf, KP, 0, 1.0, P.A1top, KP,
                                 P.A1top, KP, st));
        PROF("small_gemm", st, launch_small_gemm(ik0, ik, ik0, 1.0, P.Pm, k0, 1, P.A1top, KP, 0, 0.0, nullptr, 0, S,
                                 lds, st));
    }

    // QR of the bottom block: chunked Householder QR of A_low (+ V Z on the fly)
    std::vector<TsqrLevel> Ls = tsqr_levels(P.ts, A + k0 * lda, lda, Q + k0 * ldq, ldq);
    if (k0 > 0) {
        Ls[0].V = V + k0 * ldv;
        Ls[0].ldv = ldv;
        Ls[0].k0 = ik0;
        Ls[0].Z = P.Zperm;
        Ls[0].Nc = P.Nc;
        Ls[0].Nglob = P.Nperm;
        Ls[0].Zlp = P.Zlp;
        Ls[0].Nlp = P.Nlp;
    }
    rc = tsqr_factor(P.ts, Ls, K0P, R, ldr, st, panel);
    if (rc) return rc;

    if (k0 > 0) {
        // formation of Q: G = W^T [0; Q_] = -sum_c N_c G_c ;  N = T^{-1} G.
        // The per-chunk products go first (short, and they need more shared
        // memory than is left beside the chain below).
        PROF("chunk_prod", st, launch_chunk_prod(Ls[0].nchunk, K0P, KP, ik, P.Nc, Ls[0].Gin, Ls[0].ldg, Ls[0].gstride,
                                 P.prod, st));
        // the k x k recurrence of the level-0 formation needs neither G nor N:
        // it runs on the side stream while they are computed
        Fork& f = fork_for_thread();
        HIPCHK(hipEventRecord(f.ev0, st));
        HIPCHK(hipStreamWaitEvent(f.side, f.ev0, 0));
        rc = tsqr_kchain0(P.ts, Ls, f.side);
        if (rc) return rc;
        HIPCHK(hipEventRecord(f.ev1, f.side));
        PROF("reduce_parts", st, launch_reduce_parts(Ls[0].nchunk, (int64_t)K0P * KP, P.prod, P.Mbuf, st));
        PROF("small_gemm", st, launch_small_gemm(K0P, KP, 0, 0.0, P.Mbuf, KP, 0, P.Mbuf, KP, 0, -1.0, P.Mbuf, KP,
                                 P.Nglob, KP, st));
        PROF("trsm", st, launch_trsm_lower(ik0, ik, P.Tm, k0, 0, P.Nglob, KP, st));
        PROF("permute", st, launch_permute_b(K0P, KP, P.Nglob, P.Nperm, st));
        if (panel) PROF("pack_lowp", st, launch_pack_b_lowp(panel, K0P, KP, P.Nglob, P.Nlp, st));
        // Q_top = -(P - V_top) N
        PROF("small_gemm", st, launch_small_gemm(ik0, ik, ik0, 1.0, V, ldv, 0, P.Nglob, KP, 0, 0.0, nullptr, 0, Q, ldq,
                                 st));
        PROF("small_gemm", st, launch_small_gemm(ik0, ik, ik0, -1.0, P.Pm, k0, 0, P.Nglob, KP, 0, 1.0, Q, ldq, Q, ldq,
                                 st));
        HIPCHK(hipStreamWaitEvent(st, f.ev1, 0));
        return tsqr_rows0(P.ts, Ls, K0P, st, panel);
    }
    return tsqr_form0(P.ts, Ls, K0P, st, panel);
}

size_t two_stage_bytes(int64_t n, int64_t k0, int64_t k, int panel = 0) {
    if (k == 0) return 0;
    TwoStagePlan P;
    make_plan(n, k0, k, nullptr, P, panel);
    return P.bytes;
}

// Block Householder QR of [V, A] (Algorithm 4 over column panels of at most
// 64): the first panel by the chunked Householder QR, every later panel
// against the computed basis of the earlier ones by the generalized
// Householder step of Algorithm 1; A is the last panel.
struct HhqrPlan {
    double *Qv, *Rtmp, *Stmp;
    void* sub;
    size_t bytes;
};

void make_hhqr_plan(int64_t n, int64_t k0, int64_t k, void* ws, HhqrPlan& H) {
    Carve cv(ws);
    H.Qv = cv.take((size_t)n * std::max<int64_t>(k0, 1));
    H.Rtmp = cv.take(64 * 64);
    H.Stmp = cv.take((size_t)std::max<int64_t>(k0, 1) * 64);
    size_t sub = two_stage_bytes(n, k0, k);
    for (int64_t c = 0; c < k0; c += 64) sub = std::max(sub, two_stage_bytes(n, c, std::min<int64_t>(64, k0 - c)));
    H.sub = cv.take(sub / sizeof(double) + 1);
    H.bytes = cv.bytes();
}

}  // namespace

extern "C" {

const char* tho_version(void) { return "tho 0.1.0 (gfx950)"; }

const char* tho_last_error(void) { return last_error(); }

const char* tho_strerror(int code) {
    if (code == 0) return "success";
    if (code == THO_E_WORKSPACE) return "workspace too small";
    if (code == THO_E_HIP) return "HIP runtime error";
    if (code == THO_E_UNSUPPORTED) return "unsupported combination of arguments";
    if (code < 0) return "invalid argument";
    return "unknown code";
}

int tho_profile_enable(int on) { return prof_enable(on); }
int tho_profile_collect(void) { return prof_collect(); }
int tho_profile_reset(void) { return prof_reset(); }
int tho_profile_get(int i, char* name, int name_len, double* total_ms, int64_t* launches) {
    return prof_get(i, name, name_len, total_ms, launches);
}

int tho_two_stage_workspace(int32_t dtype, int64_t n, int64_t k0, int64_t k, const tho_opts_t* opts,
                            size_t* bytes) {
    int rc = check_common(dtype, n, k0, k);
    if (rc) return rc;
    if (!bytes) return set_err(-6, "bytes must not be NULL");
    const int panel = opts ? opts->panel : 0;
    if (panel < THO_PANEL_F64 || panel > THO_PANEL_BF16) return set_err(-5, "unknown panel precision");
    if (dtype == THO_C128) {
        if (!zsupported(k0, k)) return set_err(THO_E_UNSUPPORTED, "complex128 supports k0 <= 64, k <= 32");
        if (panel != THO_PANEL_F64) return set_err(THO_E_UNSUPPORTED, "reduced-precision panels are real only");
        *bytes = ztwo_stage_bytes(n, k0, k);
        return 0;
    }
    *bytes = two_stage_bytes(n, k0, k, panel);
    return 0;
}

int tho_two_stage(int32_t dtype, int64_t n, int64_t k0, int64_t k, const void* V_, int64_t ldv,
                  const void* A_, int64_t lda, void* Q_, int64_t ldq, void* R_, int64_t ldr, void* S_,
                  int64_t lds, const tho_opts_t* opts, void* ws, size_t ws_bytes, void* stream) {
    int rc = check_common(dtype, n, k0, k);
    if (rc) return rc;
    const int panel = opts ? opts->panel : 0;
    if (opts && (opts->p_choice != THO_P_QR || opts->flags != 0))
        return set_err(THO_E_UNSUPPORTED, "only p_choice=THO_P_QR without flags is implemented");
    if (panel < THO_PANEL_F64 || panel > THO_PANEL_BF16) return set_err(-15, "unknown panel precision");
    if (dtype == THO_C128) {
        if (!zsupported(k0, k)) return set_err(THO_E_UNSUPPORTED, "complex128 supports k0 <= 64, k <= 32");
        if (panel != THO_PANEL_F64) return set_err(THO_E_UNSUPPORTED, "reduced-precision panels are real only");
        if (k == 0) return 0;
        if ((rc = check_io(k0, k, V_, ldv, A_, lda, Q_, ldq, R_, ldr, S_, lds))) return rc;
        for (const void* p : {V_, A_, (const void*)Q_, (const void*)R_, (const void*)S_})
            if (p && ((uintptr_t)p & 15)) return set_err(-5, "complex matrices must be 16-byte aligned");
        if (!ws) return set_err(-16, "workspace is NULL");
        if (ws_bytes < ztwo_stage_bytes(n, k0, k)) return set_err(THO_E_WORKSPACE, "workspace too small");
        return run_ztwo_stage(n, k0, k, (const dcplx*)V_, ldv, (const dcplx*)A_, lda, (dcplx*)Q_, ldq, (dcplx*)R_,
                              ldr, (dcplx*)S_, lds, ws, (hipStream_t)stream);
    }
    if (k == 0) return 0;
    rc = check_io(k0, k, V_, ldv, A_, lda, Q_, ldq, R_, ldr, S_, lds);
    if (rc) return rc;
    if (!ws) return set_err(-16, "workspace is NULL");
    if (ws_bytes < two_stage_bytes(n, k0, k, panel)) return set_err(THO_E_WORKSPACE, "workspace too small");
    return run_two_stage(n, k0, k, (const double*)V_, ldv, (const double*)A_, lda, (double*)Q_, ldq, (double*)R_, ldr,
                         (double*)S_, lds, ws, (hipStream_t)stream, panel);
}

int tho_hhqr_full_workspace(int32_t dtype, int64_t n, int64_t k0, int64_t k, const tho_opts_t* opts, size_t* bytes) {
    int rc = check_common(dtype, n, k0, k);
    if (rc) return rc;
    if (!bytes) return set_err(-6, "bytes must not be NULL");
    (void)opts;
    if (k == 0) { *bytes = 0; return 0; }
    if (dtype == THO_C128) {
        if (!zsupported(k0, k)) return set_err(THO_E_UNSUPPORTED, "complex128 supports k0 <= 64, k <= 32");
        *bytes = zhhqr_bytes(n, k0, k);
        return 0;
    }
    HhqrPlan H;
    make_hhqr_plan(n, k0, k, nullptr, H);
    *bytes = H.bytes;
    return 0;
}

int tho_hhqr_full(int32_t dtype, int64_t n, int64_t k0, int64_t k, const void* V_, int64_t ldv, const void* A_,
                  int64_t lda, void* Q_, int64_t ldq, void* R_, int64_t ldr, void* S_, int64_t lds,
                  const tho_opts_t* opts, void* ws, size_t ws_bytes, void* stream) {
    int rc = check_common(dtype, n, k0, k);
    if (rc) return rc;
    if (opts && (opts->panel != THO_PANEL_F64 || opts->flags != 0))
        return set_err(THO_E_UNSUPPORTED, "tho_hhqr_full supports panel=THO_PANEL_F64 only");
    if (dtype == THO_C128 && !zsupported(k0, k))
        return set_err(THO_E_UNSUPPORTED, "complex128 supports k0 <= 64, k <= 32");
    if (k == 0) return 0;
    if ((rc = check_io(k0, k, V_, ldv, A_, lda, Q_, ldq, R_, ldr, S_, lds))) return rc;
    if (!ws) return set_err(-16, "workspace is NULL");
    if (dtype == THO_C128) {
        if (ws_bytes < zhhqr_bytes(n, k0, k)) return set_err(THO_E_WORKSPACE, "workspace too small");
        return run_zhhqr(n, k0, k, (const dcplx*)V_, ldv, (const dcplx*)A_, lda, (dcplx*)Q_, ldq, (dcplx*)R_, ldr,
                         (dcplx*)S_, lds, ws, (hipStream_t)stream);
    }
    HhqrPlan H;
    make_hhqr_plan(n, k0, k, nullptr, H);
    if (ws_bytes < H.bytes) return set_err(THO_E_WORKSPACE, "workspace too small");
    make_hhqr_plan(n, k0, k, ws, H);
    hipStream_t st = (hipStream_t)stream;
    const double* V = (const double*)V_;
    // panels of V: Q_B[:, c:c+w] and R_B[c:c+w, c:c+w] (R_B's V block is not returned)
    for (int64_t c = 0; c < k0; c += 64) {
        const int64_t w = std::min<int64_t>(64, k0 - c);
        rc = run_two_stage(n, c, w, H.Qv, k0, V + c, ldv, H.Qv + c, k0, H.Rtmp, 64, H.Stmp, 64, H.sub, st);
        if (rc) return rc;
    }
    // last panel A: Q = Q_B[:, k0:], R = R_B[k0:, k0:], S = R_B[:k0, k0:]
    return run_two_stage(n, k0, k, H.Qv, k0, (const double*)A_, lda, (double*)Q_, ldq, (double*)R_, ldr, (double*)S_,
                         lds, H.sub, st);
}

}  // extern "C"
