// C ABI of libtho: argument validation, workspace layout and the launch
// sequence of the two-stage Householder orthogonalization (Algorithm 1 of
// He & Shao, any of the three choices of P of §3.2) on one HIP stream.  No host
// synchronization and no device allocation happen here.
#include <algorithm>
#include <climits>

#include "tho_host.h"

using namespace tho;

namespace {

struct TwoStagePlan {
    int KP, K0P;
    XtyPlan xp;
    TsqrPlan ts;
    double *part, *Cbuf, *Pm, *Tm, *Zbuf, *A1top, *Mbuf, *Nglob, *Nc, *prod, *Zperm, *Nperm;
    double *F2, *pws;  // first / third choice of P: second factor of T, polar workspace
    double *Zlp, *Nlp;  // reduced-precision panels only
    size_t bytes;
};

void make_plan(int64_t n, int64_t k0, int64_t k, void* ws, TwoStagePlan& P, int panel = 0, int pchoice = 0) {
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
        P.F2 = (pchoice == THO_P_MLU) ? cv.take((size_t)k0 * k0) : nullptr;
        P.pws = (pchoice == THO_P_POLAR) ? cv.take(pchoice_ws_doubles((int)k0)) : nullptr;
        P.Zlp = P.Nlp = nullptr;
        if (panel != 0) {
            const size_t lb = lowp_pack_bytes(panel, P.K0P, P.KP) / sizeof(double) + 1;
            P.Zlp = cv.take(lb);
            P.Nlp = cv.take(lb);
        }
    } else {
        P.part = P.Cbuf = P.Pm = P.Tm = P.Zbuf = P.A1top = P.Mbuf = P.Nglob = P.Nc = P.prod = nullptr;
        P.Zperm = P.Nperm = P.Zlp = P.Nlp = nullptr;
        P.F2 = P.pws = nullptr;
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

// Do two row-major blocks (rows x cols elements of esz bytes, row stride ld
// elements) share an element?  Exact when the row strides are equal and
// the second block does not wrap around a row of the first; otherwise the
// answer is "yes" whenever their address ranges meet.
bool blocks_overlap(const void* p1, int64_t r1, int64_t c1, int64_t ld1, const void* p2, int64_t r2, int64_t c2,
                    int64_t ld2, int64_t esz) {
    if (!p1 || !p2 || r1 <= 0 || c1 <= 0 || r2 <= 0 || c2 <= 0) return false;
    const uintptr_t a0 = (uintptr_t)p1, a1 = a0 + (uintptr_t)(((r1 - 1) * ld1 + c1) * esz);
    const uintptr_t b0 = (uintptr_t)p2, b1 = b0 + (uintptr_t)(((r2 - 1) * ld2 + c2) * esz);
    if (a1 <= b0 || b1 <= a0) return false;
    if (ld1 != ld2) return true;
    const bool swap = b0 < a0;
    const uintptr_t lo = swap ? b0 : a0, hi = swap ? a0 : b0;
    const int64_t rlo = swap ? r2 : r1, clo = swap ? c2 : c1, rhi = swap ? r1 : r2, chi = swap ? c1 : c2;
    if ((hi - lo) % (uintptr_t)esz) return true;
    const int64_t d = (int64_t)((hi - lo) / (uintptr_t)esz);
    const int64_t dr = d / ld1, dc = d % ld1;
    if (dc + chi > ld1) return true;  // the later block wraps into the next row
    const bool rows_meet = dr < rlo && dr + rhi > 0;
    const bool cols_meet = dc < clo && dc + chi > 0;
    return rows_meet && cols_meet;
}

// Outputs Q (arg 9), R (11), S (13) must not share elements with the inputs
// or each other; returns -i for the first output that does.
int check_alias(int64_t n, int64_t k0, int64_t k, int64_t esz, const void* V, int64_t ldv, const void* A,
                int64_t lda, const void* Q, int64_t ldq, const void* R, int64_t ldr, const void* S, int64_t lds) {
    struct Blk { const void* p; int64_t r, c, ld; };
    const Blk v{V, n, k0, ldv}, a{A, n, k, lda}, q{Q, n, k, ldq}, r{R, k, k, ldr}, s{S, k0, k, lds};
    auto ov = [&](const Blk& x, const Blk& y) { return blocks_overlap(x.p, x.r, x.c, x.ld, y.p, y.r, y.c, y.ld, esz); };
    if (ov(q, v) || ov(q, a)) return set_err(-9, "Q overlaps an input");
    if (ov(r, v) || ov(r, a) || ov(r, q)) return set_err(-11, "R overlaps an input or Q");
    if (ov(s, v) || ov(s, a) || ov(s, q) || ov(s, r)) return set_err(-13, "S overlaps an input, Q or R");
    return 0;
}
}  // namespace tho

namespace tho {

// P and the factors of T for the chosen P (§3.2), one workgroup on `s`, for
// the k0 x k0 top block at V (ld ldv); Pm, Tm, F2 are k0 x k0 with ld k0:
//   first choice  (THO_P_MLU)    Tm = P L, F2 = U^T with P - V_top = L U
//   second choice (THO_P_QR)     Tm = T = I + R1^T (lower)
//   third choice  (THO_P_POLAR)  Tm = C, T = I + M = C C^T (pws: polar workspace)
int p_and_t(int pchoice, int k0, const double* V, int64_t ldv, double* Pm, double* Tm, double* F2, double* pws,
            hipStream_t s) {
    if (pchoice == THO_P_MLU) PROF("mlu_top", s, launch_mlu_top(k0, V, ldv, Pm, Tm, F2, s));
    else if (pchoice == THO_P_POLAR) PROF("polar_top", s, launch_polar_top(k0, V, ldv, Pm, Tm, pws, s));
    else PROF("qr_top", s, launch_qr_top(k0, V, ldv, Pm, Tm, s));
    return 0;
}

// B <- T^{-T} B (k0 x k columns of B, ld ldb).  First choice:
// T^T = P L U; second: T lower; third: T = C C^T.
int solve_tt(int pchoice, int k0, int k, const double* Tm, const double* F2, double* B, int64_t ldb, hipStream_t st) {
    if (pchoice == THO_P_MLU) {
        PROF("trsm", st, launch_trsm_lower(k0, k, Tm, k0, 0, B, ldb, st));
        PROF("trsm", st, launch_trsm_lower(k0, k, F2, k0, 1, B, ldb, st));
    } else if (pchoice == THO_P_POLAR) {
        PROF("trsm", st, launch_trsm_lower(k0, k, Tm, k0, 0, B, ldb, st));
        PROF("trsm", st, launch_trsm_lower(k0, k, Tm, k0, 1, B, ldb, st));
    } else {
        PROF("trsm", st, launch_trsm_lower(k0, k, Tm, k0, 1, B, ldb, st));
    }
    return 0;
}

// B <- T^{-1} B.  First choice: T = U^T (L^T P).
int solve_t(int pchoice, int k0, int k, const double* Tm, const double* F2, double* B, int64_t ldb, hipStream_t st) {
    if (pchoice == THO_P_MLU) {
        PROF("trsm", st, launch_trsm_lower(k0, k, F2, k0, 0, B, ldb, st));
        PROF("trsm", st, launch_trsm_lower(k0, k, Tm, k0, 1, B, ldb, st));
    } else if (pchoice == THO_P_POLAR) {
        PROF("trsm", st, launch_trsm_lower(k0, k, Tm, k0, 0, B, ldb, st));
        PROF("trsm", st, launch_trsm_lower(k0, k, Tm, k0, 1, B, ldb, st));
    } else {
        PROF("trsm", st, launch_trsm_lower(k0, k, Tm, k0, 0, B, ldb, st));
    }
    return 0;
}

}  // namespace tho

namespace {

// Launch sequence of Algorithm 1 on validated arguments; ws holds at least
// two_stage_bytes(n, k0, k, panel, pchoice).
int run_two_stage(int64_t n, int64_t k0, int64_t k, const double* V, int64_t ldv, const double* A, int64_t lda,
                  double* Q, int64_t ldq, double* R, int64_t ldr, double* S, int64_t lds, void* ws,
                  hipStream_t st, int panel = 0, int pchoice = THO_P_QR) {
    int rc = 0;
    if (k0 == 0) panel = 0;
    TwoStagePlan P;
    make_plan(n, k0, k, ws, P, panel, pchoice);
    const int KP = P.KP, K0P = P.K0P;
    const int ik = (int)k, ik0 = (int)k0;
    const size_t nk = (size_t)std::max(K0P, 16) * KP;

    if (k0 > 0) {
        // P and T (§3.2; second choice: V_top = Q1 R1, P = -Q1, T = I + R1^T)
        // on a side stream, concurrently with the reduction C = V^T A over
        // all n rows (update of A); joined before the first use of P and T
        Fork& f = fork_for_thread();
        if (!f.ok) return set_err(THO_E_HIP, "could not create the side stream");
        HIPCHK(hipEventRecord(f.ev0, st));
        HIPCHK(hipStreamWaitEvent(f.side, f.ev0, 0));
        if ((rc = p_and_t(pchoice, ik0, V, ldv, P.Pm, P.Tm, P.F2, P.pws, f.side))) return rc;
        HIPCHK(hipEventRecord(f.ev1, f.side));
        rc = xty(P.xp, n, V, ldv, ik0, A, lda, ik, P.part, P.Cbuf, st, "xty_partial", panel);
        if (rc) return rc;
        HIPCHK(hipStreamWaitEvent(st, f.ev1, 0));
        // W^T A = P^T A_top - C ;  Z = T^{-T} (W^T A)
        PROF("fill", st, fill(P.Zbuf, (int64_t)nk, 0.0, st));
        PROF("small_gemm", st, launch_small_gemm(ik0, ik, ik0, 1.0, P.Pm, k0, 1, A, lda, 0, -1.0, P.Cbuf, KP, P.Zbuf,
                                 KP, st));
        if ((rc = solve_tt(pchoice, ik0, ik, P.Tm, P.F2, P.Zbuf, KP, st))) return rc;
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
        if ((rc = solve_t(pchoice, ik0, ik, P.Tm, P.F2, P.Nglob, KP, st))) return rc;
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

size_t two_stage_bytes(int64_t n, int64_t k0, int64_t k, int panel = 0, int pchoice = THO_P_QR) {
    if (k == 0) return 0;
    TwoStagePlan P;
    make_plan(n, k0, k, nullptr, P, panel, pchoice);
    return P.bytes;
}

}  // namespace

namespace tho {
// Householder QR of an m x k block (k <= 64) with nonnegative diag(R): the
// k0 = 0 case of the two-stage launch sequence.  Q may equal X.
size_t plain_qr_bytes(int64_t m, int64_t k) { return two_stage_bytes(m, 0, k); }
int run_plain_qr(int64_t m, int64_t k, const double* X, int64_t ldx, double* Q, int64_t ldq, double* R, int64_t ldr,
                 void* ws, hipStream_t st) {
    return run_two_stage(m, 0, k, nullptr, 0, X, ldx, Q, ldq, R, ldr, nullptr, 0, ws, st);
}
}  // namespace tho

namespace {

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

namespace {

// Leading part of tho_two_stage's workspace: the info word (256 bytes) and,
// with THO_CHECK_VORTH and k0 > 0, the split-n partials and the two column
// blocks of the Gram of V (real view for complex).
constexpr size_t INFO_BYTES = 256;

struct CheckPlan {
    XtyPlan xp;
    double *part = nullptr, *G0 = nullptr, *G1 = nullptr;
    size_t bytes = INFO_BYTES;
};

void make_check_plan(int64_t n, int64_t k0, int flags, int w, void* ws, CheckPlan& C) {
    C = CheckPlan();
    if (!(flags & THO_CHECK_VORTH) || k0 == 0) return;
    Carve cv(ws ? (char*)ws + INFO_BYTES : nullptr);
    C.xp = xty_plan(n);
    const int p = (int)(w * k0);
    C.part = cv.take((size_t)C.xp.nblk * k0p_of(p) * 64);
    C.G0 = cv.take((size_t)k0p_of(p) * 64);
    C.G1 = cv.take((size_t)k0p_of(p) * 64);
    C.bytes = INFO_BYTES + cv.bytes();
}

// ||V^* V - I||_F > THO_VORTH_TOL -> info 3, from the Gram of V (as a real
// n x w k0 matrix) in two column blocks of at most 64.
int vorth_check(int64_t n, int64_t k0, int w, const double* V, int64_t ldv, const CheckPlan& C, int* info,
                hipStream_t st) {
    const int p = (int)(w * k0);
    const int q0 = std::min(p, 64), q1 = p - q0;
    int rc = xty(C.xp, n, V, w * ldv, p, V, w * ldv, q0, C.part, C.G0, st, "xty_gram");
    if (rc) return rc;
    if (q1 > 0 && (rc = xty(C.xp, n, V, w * ldv, p, V + 64, w * ldv, q1, C.part, C.G1, st, "xty_gram"))) return rc;
    // xty writes k0p_of(p) x kp_of(q) blocks with row stride kp_of(q)
    PROF("vorth_check", st, launch_vorth_check((int)k0, w == 2, C.G0, kp_of(q0), C.G1, q1 > 0 ? kp_of(q1) : 16,
                                               THO_VORTH_TOL, info, st));
    return 0;
}

}  // namespace

extern "C" {

const char* tho_version(void) { return "tho 0.2.0 (gfx950)"; }

int tho_get_info(const void* ws, int32_t* host_info) {
    if (!host_info) return set_err(-2, "host_info must not be NULL");
    const void* src = ws;
    if (!src) {
        int rc = noalloc_scratch(&src);
        if (rc) return rc;
    }
    int32_t v = 0;
    HIPCHK(hipMemcpy(&v, src, sizeof(v), hipMemcpyDeviceToHost));
    *host_info = (v == INT32_MAX) ? 0 : v;
    return 0;
}

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
    const int pchoice = opts ? opts->p_choice : THO_P_QR;
    if (panel < THO_PANEL_F64 || panel > THO_PANEL_BF16) return set_err(-5, "unknown panel precision");
    if (pchoice < THO_P_QR || pchoice > THO_P_POLAR) return set_err(-5, "unknown choice of P");
    const int flags = opts ? opts->flags : 0;
    if (flags & ~(THO_CHECK_FINITE | THO_CHECK_VORTH)) return set_err(-5, "unknown flags");
    CheckPlan C;
    if (dtype == THO_C128) {
        if (!zsupported(k0, k)) return set_err(THO_E_UNSUPPORTED, "complex128 supports k0 <= 64, k <= 32");
        if (panel != THO_PANEL_F64) return set_err(THO_E_UNSUPPORTED, "reduced-precision panels are real only");
        if (pchoice != THO_P_QR) return set_err(THO_E_UNSUPPORTED, "complex128 uses the second choice of P only");
        make_check_plan(n, k0, flags, 2, nullptr, C);
        *bytes = (k == 0) ? 0 : C.bytes + ztwo_stage_bytes(n, k0, k);
        return 0;
    }
    make_check_plan(n, k0, flags, 1, nullptr, C);
    *bytes = (k == 0) ? 0 : C.bytes + two_stage_bytes(n, k0, k, panel, pchoice);
    return 0;
}

int tho_two_stage(int32_t dtype, int64_t n, int64_t k0, int64_t k, const void* V_, int64_t ldv,
                  const void* A_, int64_t lda, void* Q_, int64_t ldq, void* R_, int64_t ldr, void* S_,
                  int64_t lds, const tho_opts_t* opts, void* ws, size_t ws_bytes, void* stream) {
    int rc = check_common(dtype, n, k0, k);
    if (rc) return rc;
    const int panel = opts ? opts->panel : 0;
    const int pchoice = opts ? opts->p_choice : THO_P_QR;
    const int flags = opts ? opts->flags : 0;
    if (panel < THO_PANEL_F64 || panel > THO_PANEL_BF16) return set_err(-15, "unknown panel precision");
    if (pchoice < THO_P_QR || pchoice > THO_P_POLAR) return set_err(-15, "unknown choice of P");
    if (flags & ~(THO_CHECK_FINITE | THO_CHECK_VORTH)) return set_err(-15, "unknown flags");
    const bool cplx = dtype == THO_C128;
    const int w = cplx ? 2 : 1;
    if (cplx) {
        if (!zsupported(k0, k)) return set_err(THO_E_UNSUPPORTED, "complex128 supports k0 <= 64, k <= 32");
        if (panel != THO_PANEL_F64) return set_err(THO_E_UNSUPPORTED, "reduced-precision panels are real only");
        if (pchoice != THO_P_QR) return set_err(THO_E_UNSUPPORTED, "complex128 uses the second choice of P only");
    }
    if (k == 0) return 0;
    if ((rc = check_io(k0, k, V_, ldv, A_, lda, Q_, ldq, R_, ldr, S_, lds))) return rc;
    if (cplx)
        for (const void* p : {V_, A_, (const void*)Q_, (const void*)R_, (const void*)S_})
            if (p && ((uintptr_t)p & 15)) return set_err(-5, "complex matrices must be 16-byte aligned");
    if ((rc = check_alias(n, k0, k, 8 * w, V_, ldv, A_, lda, Q_, ldq, R_, ldr, S_, lds))) return rc;
    if (!ws) return set_err(-16, "workspace is NULL");
    CheckPlan C;
    make_check_plan(n, k0, flags, w, nullptr, C);
    const size_t run_bytes = cplx ? ztwo_stage_bytes(n, k0, k) : two_stage_bytes(n, k0, k, panel, pchoice);
    if (ws_bytes < C.bytes + run_bytes) return set_err(THO_E_WORKSPACE, "workspace too small");
    make_check_plan(n, k0, flags, w, ws, C);
    hipStream_t st = (hipStream_t)stream;
    int* info = (int*)ws;
    void* rws = (char*)ws + C.bytes;
    PROF("info_reset", st, launch_info_reset(info, st));
    if ((flags & THO_CHECK_VORTH) && k0 > 0 && (rc = vorth_check(n, k0, w, (const double*)V_, ldv, C, info, st)))
        return rc;
    if (cplx)
        rc = run_ztwo_stage(n, k0, k, (const dcplx*)V_, ldv, (const dcplx*)A_, lda, (dcplx*)Q_, ldq, (dcplx*)R_, ldr,
                            (dcplx*)S_, lds, rws, st);
    else
        rc = run_two_stage(n, k0, k, (const double*)V_, ldv, (const double*)A_, lda, (double*)Q_, ldq, (double*)R_,
                           ldr, (double*)S_, lds, rws, st, panel, pchoice);
    if (rc) return rc;
    if (flags & THO_CHECK_FINITE)
        PROF("check_finite", st, launch_check_finite((int)k0, (int)k, cplx, (const double*)S_, lds,
                                                     (const double*)R_, ldr, info, st));
    return 0;
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
    if (opts && (opts->panel != THO_PANEL_F64 || opts->flags != 0 || opts->p_choice != THO_P_QR))
        return set_err(THO_E_UNSUPPORTED, "tho_hhqr_full supports the default options only");
    if (dtype == THO_C128 && !zsupported(k0, k))
        return set_err(THO_E_UNSUPPORTED, "complex128 supports k0 <= 64, k <= 32");
    if (k == 0) return 0;
    if ((rc = check_io(k0, k, V_, ldv, A_, lda, Q_, ldq, R_, ldr, S_, lds))) return rc;
    if ((rc = check_alias(n, k0, k, dtype == THO_C128 ? 16 : 8, V_, ldv, A_, lda, Q_, ldq, R_, ldr, S_, lds)))
        return rc;
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
