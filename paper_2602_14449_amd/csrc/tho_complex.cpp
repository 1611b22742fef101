// Complex (complex128) two-stage orthogonalization, BCGS and full
// Householder QR: Algorithm 1 with the second choice of P in complex
// arithmetic (conjugate transposes throughout).
//
// Panel products run on the real FP64 MFMA kernels through real views of the
// interleaved data: a complex n x p matrix is a real n x 2p matrix whose
// columns alternate re, im.
//   X^H Y:      the real reduction X_ri^T Y_ri (2p x 2q) and a re/im combine;
//   Y + X B:    the real row-streaming product with B in 2 x 2 real block
//               form [[br, bi], [-bi, br]].
// The Householder QR of the bottom block and the formation of Q_ are complex
// kernels (k_complex.hip); unlike the real path the update A + V Z and the
// term V N are separate passes over the rows.
#include <algorithm>

#include "tho_host.h"

using namespace tho;

namespace {

constexpr int ZMAX_K0 = 64, ZMAX_K = 32;

struct ZTsqrPlan {
    int64_t m = 0;
    int k = 0, KP = 16;
    std::vector<LevelPlan> lv;
    dcplx *Rtop = nullptr, *G0 = nullptr;
    std::vector<dcplx*> Tt, stack;
};

dcplx* ztake(Carve& cv, size_t n) { return (dcplx*)cv.take(2 * n); }

void ztsqr_plan(int64_t m0, int k, Carve& cv, ZTsqrPlan& T) {
    T.m = m0;
    T.k = k;
    T.KP = k <= 16 ? 16 : 32;
    T.lv.clear();
    const int tb = ztsqr_tile_rows(T.KP);
    int64_t m = m0;
    for (int level = 0;; level++) {
        int64_t nc = cdiv(m, tb);
        if (level == 0) nc = std::min<int64_t>(nc, 512);
        nc = std::max<int64_t>(1, std::min<int64_t>(nc, m / std::max(1, k)));
        T.lv.push_back({m, (int)nc, (int)cdiv(cdiv(m, nc), tb)});
        if (nc == 1) break;
        m = nc * k;
    }
    const size_t kk = (size_t)T.KP * T.KP;
    T.Rtop = ztake(cv, kk);
    T.G0 = ztake(cv, kk);
    T.Tt.assign(T.lv.size(), nullptr);
    T.stack.assign(T.lv.size(), nullptr);
    for (size_t l = 0; l < T.lv.size(); l++) {
        T.Tt[l] = ztake(cv, (size_t)T.lv[l].nchunk * T.lv[l].maxtiles * kk);
        if (l >= 1) T.stack[l] = ztake(cv, (size_t)T.lv[l].m * T.KP);
    }
}

std::vector<ZLevel> ztsqr_levels(const ZTsqrPlan& T, const dcplx* X, int64_t ldx, dcplx* Y, int64_t ldy) {
    const int nl = (int)T.lv.size();
    std::vector<ZLevel> Ls(nl);
    for (int l = 0; l < nl; l++) {
        ZLevel& L = Ls[l];
        std::memset(&L, 0, sizeof(L));
        L.m = T.lv[l].m;
        L.k = T.k;
        L.nchunk = T.lv[l].nchunk;
        L.maxtiles = T.lv[l].maxtiles;
        L.X = l == 0 ? X : T.stack[l];
        L.ldx = l == 0 ? ldx : T.KP;
        L.Y = l == 0 ? Y : T.stack[l];
        L.ldy = l == 0 ? ldy : T.KP;
        L.Tt = T.Tt[l];
        L.Rnext = (l + 1 < nl) ? T.stack[l + 1] : T.Rtop;
        L.ldrn = T.KP;
        L.Gin = (l + 1 < nl) ? T.stack[l + 1] : T.G0;
        L.ldg = T.KP;
        L.gstride = (l + 1 < nl) ? T.k : 0;
    }
    return Ls;
}

// Householder QR of X (m x k) into explicit Q_ (in Y) and R (nonnegative
// real diagonal); Y may equal X.
// Optional V term of level 0 (Algorithm 1): the leaf factors A + V Z (Z in
// B-operand order) and leaves M_c = Q_chunk^H V_chunk per chunk in Nc.
struct ZFuse {
    const dcplx* V = nullptr;
    int64_t ldv = 0;
    int k0 = 0, K0P = 0;
    const dcplx* Zp = nullptr;
    dcplx* Nc = nullptr;
};

int ztsqr(const ZTsqrPlan& T, const dcplx* X, int64_t ldx, dcplx* Y, int64_t ldy, dcplx* R, int64_t ldr,
          hipStream_t st, const ZFuse* fz = nullptr, std::vector<ZLevel>* out_levels = nullptr, bool form0 = true) {
    std::vector<ZLevel> Ls = ztsqr_levels(T, X, ldx, Y, ldy);
    const int nl = (int)Ls.size();
    {
        const ZLevel& z = Ls[0];
        ZRLevel L0{};
        L0.m = z.m;
        L0.k = z.k;
        L0.nchunk = z.nchunk;
        L0.maxtiles = z.maxtiles;
        L0.X = z.X;
        L0.ldx = z.ldx;
        L0.Y = z.Y;
        L0.ldy = z.ldy;
        L0.Tt = z.Tt;
        L0.Rnext = z.Rnext;
        L0.ldrn = z.ldrn;
        int k0p = 0;
        if (fz && fz->k0 > 0) {
            L0.V = fz->V;
            L0.ldv = fz->ldv;
            L0.k0 = fz->k0;
            L0.Zp = fz->Zp;
            L0.Nc = fz->Nc;
            k0p = fz->K0P;
        }
        PROF("zleaf_l0", st, launch_zleaf_rt(T.KP, k0p, L0, st));
    }
    for (int l = 1; l < nl; l++) {
        const ZLevel& z = Ls[l];
        ZRLevel Lu{};
        Lu.m = z.m;
        Lu.k = z.k;
        Lu.nchunk = z.nchunk;
        Lu.maxtiles = z.maxtiles;
        Lu.X = z.X;
        Lu.ldx = z.ldx;
        Lu.Y = z.Y;
        Lu.ldy = z.ldy;
        Lu.Tt = z.Tt;
        Lu.Rnext = z.Rnext;
        Lu.ldrn = z.ldrn;
        PROF("zleaf_up", st, launch_zleaf_rt(T.KP, 0, Lu, st));
    }
    if (out_levels) *out_levels = Ls;
    PROF("zfinish_r", st, launch_zfinish_r(T.k, T.KP, T.Rtop, T.KP, R, ldr, T.G0, st));
    for (int l = nl - 1; l >= (form0 ? 0 : 1); l--)
        PROF(l == 0 ? "zform_l0" : "zform_up", st, launch_zform(T.KP, Ls[l], st));
    return 0;
}

// Complex reduction out (p x q, ld ldo) = sign * X^H Y over nrows rows.
struct ZXty {
    XtyPlan xp;
    double *part, *raw;
    int P2, Q2;  // padded real view sizes
};

void zxty_plan(int64_t nrows, int p, int q, Carve& cv, ZXty& Z) {
    Z.xp = xty_plan(nrows);
    Z.P2 = k0p_of(2 * p);
    Z.Q2 = kp_of(2 * q);
    Z.part = cv.take((size_t)Z.xp.nblk * Z.P2 * Z.Q2);
    Z.raw = cv.take((size_t)Z.P2 * Z.Q2);
}

int zxty(const ZXty& Z, int64_t nrows, const dcplx* X, int64_t ldx, int p, const dcplx* Y, int64_t ldy, int q,
         double sign, dcplx* out, int64_t ldo, hipStream_t st) {
    int rc = xty(Z.xp, nrows, (const double*)X, 2 * ldx, 2 * p, (const double*)Y, 2 * ldy, 2 * q, Z.part, Z.raw, st,
                 "xty_partial");
    if (rc) return rc;
    PROF("zcombine", st, launch_zcombine(p, q, Z.raw, Z.Q2, sign, out, ldo, st));
    return 0;
}

// Out (nrows x q) = X + Y B with complex B (p x q, ld ldb) scaled by sign.
struct ZRows {
    double *exp, *pk;
};

void zrows_plan(int p, int q, Carve& cv, ZRows& Z) {
    Z.exp = cv.take((size_t)4 * std::max(p, 1) * std::max(q, 1));
    Z.pk = cv.take((size_t)k0p_of(2 * p) * rows_gemm_qp(2 * q) + 64);
}

int zrows(const ZRows& Z, int64_t nrows, const dcplx* X, int64_t ldx, dcplx* Out, int64_t ldo, const dcplx* Y,
          int64_t ldy, int p, const dcplx* B, int64_t ldb, int q, double sign, hipStream_t st) {
    const int kpad = k0p_of(2 * p), qp = rows_gemm_qp(2 * q);
    PROF("zexpand", st, launch_zexpand(p, q, B, ldb, sign, Z.exp, st));
    PROF("pack_b", st, launch_pack_b(2 * p, 2 * q, Z.exp, 2 * q, 0, 1.0, kpad, qp, Z.pk, st));
    RowsGemm g{};
    g.nrows = nrows;
    g.X = (const double*)X;
    g.ldx = 2 * ldx;
    g.Out = (double*)Out;
    g.ldo = 2 * ldo;
    g.q = 2 * q;
    g.nterm = 1;
    g.t[0] = {(const double*)Y, 2 * ldy, 2 * p, kpad, Z.pk};
    PROF("rows_gemm", st, launch_rows_gemm(g, st));
    return 0;
}

struct ZPlan {
    ZTsqrPlan ts;
    ZXty xa;
    dcplx *Pm, *Tm, *C, *Z, *A1t, *N;
    dcplx *Zp, *Nc, *prod, *Gsum;  // fused level 0: permuted Z, chunk products, their reduction
    dcplx *Cfin, *Np;              // level-0 formation: final C per chunk, permuted N
    int K0P;
    size_t bytes;
};

void make_zplan(int64_t n, int64_t k0, int64_t k, void* ws, ZPlan& P) {
    Carve cv(ws);
    ztsqr_plan(n - k0, (int)k, cv, P.ts);
    P.Pm = P.Tm = P.C = P.Z = P.A1t = P.N = nullptr;
    P.Zp = P.Nc = P.prod = P.Gsum = P.Cfin = P.Np = nullptr;
    P.K0P = (int)k0p_of(k0);
    if (k0 > 0) {
        const int KP = P.ts.KP, K0P = P.K0P;
        const int nc0 = P.ts.lv[0].nchunk;
        zxty_plan(n, (int)k0, (int)k, cv, P.xa);
        P.Pm = ztake(cv, (size_t)k0 * k0);
        P.Tm = ztake(cv, (size_t)k0 * k0);
        P.C = ztake(cv, (size_t)k0 * k);
        P.Z = ztake(cv, (size_t)k0 * k);
        P.A1t = ztake(cv, (size_t)k0 * k);
        P.N = ztake(cv, (size_t)k0 * k);
        P.Zp = ztake(cv, (size_t)(K0P / 4) * (KP / 16) * 64);
        P.Nc = ztake(cv, (size_t)nc0 * KP * K0P);
        P.prod = ztake(cv, (size_t)nc0 * K0P * KP);
        P.Gsum = ztake(cv, (size_t)K0P * KP);
        P.Cfin = ztake(cv, (size_t)nc0 * KP * KP);
        P.Np = ztake(cv, (size_t)(K0P / 4) * (KP / 16) * 64);
    }
    P.bytes = cv.bytes();
}

}  // namespace

namespace tho {

bool zsupported(int64_t k0, int64_t k) { return k0 <= ZMAX_K0 && k <= ZMAX_K; }

size_t ztwo_stage_bytes(int64_t n, int64_t k0, int64_t k) {
    if (k == 0) return 0;
    ZPlan P;
    make_zplan(n, k0, k, nullptr, P);
    return P.bytes;
}

int run_ztwo_stage(int64_t n, int64_t k0, int64_t k, const dcplx* V, int64_t ldv, const dcplx* A, int64_t lda,
                   dcplx* Q, int64_t ldq, dcplx* R, int64_t ldr, dcplx* S, int64_t lds, void* ws, hipStream_t st) {
    int rc = 0;
    ZPlan P;
    make_zplan(n, k0, k, ws, P);
    const int ik = (int)k, ik0 = (int)k0;
    const int64_t m = n - k0;
    const dcplx* X0 = A + k0 * lda;  // bottom block, or its update
    int64_t ldx0 = lda;
    if (k0 > 0) {
        // P = -Q1, T = I + R1^H from V_top = Q1 R1 (real diag R1 >= 0), on a
        // side stream concurrently with the reduction V^H A over all n rows;
        // joined before the first use of P and T
        Fork& f = fork_for_thread();
        if (!f.ok) return set_err(THO_E_HIP, "could not create the side stream");
        HIPCHK(hipEventRecord(f.ev0, st));
        HIPCHK(hipStreamWaitEvent(f.side, f.ev0, 0));
        PROF("zqr_top", f.side, launch_zqr_top(ik0, V, ldv, P.Pm, P.Tm, f.side));
        HIPCHK(hipEventRecord(f.ev1, f.side));
        // W^H A = P^H A_top - V^H A ;  Z = T^{-H} W^H A
        if ((rc = zxty(P.xa, n, V, ldv, ik0, A, lda, ik, 1.0, P.C, k, st))) return rc;
        HIPCHK(hipStreamWaitEvent(st, f.ev1, 0));
        PROF("zgemm", st, launch_zgemm(ik0, ik, ik0, 1, 0, P.Pm, k0, 2, A, lda, 0, -1, 0, P.C, k, P.Z, k, st));
        PROF("ztrsm", st, launch_ztrsm(ik0, ik, P.Tm, k0, 2, P.Z, k, st));
        // A1_top = A_top - (P - V_top) Z ;  S = P^H A1_top
        PROF("zgemm", st, launch_zgemm(ik0, ik, ik0, -1, 0, P.Pm, k0, 0, P.Z, k, 0, 1, 0, A, lda, P.A1t, k, st));
        PROF("zgemm", st, launch_zgemm(ik0, ik, ik0, 1, 0, V, ldv, 0, P.Z, k, 0, 1, 0, P.A1t, k, P.A1t, k, st));
        PROF("zgemm", st, launch_zgemm(ik0, ik, ik0, 1, 0, P.Pm, k0, 2, P.A1t, k, 0, 0, 0, nullptr, 0, S, lds, st));
        // Z in the B-operand order of the fused update A1_low = A_low + V_low Z
        PROF("zpermute", st, launch_zpermute_b(P.K0P, P.ts.KP, ik0, ik, P.Z, k, P.Zp, st));
    }
    // A1_low = Q_ R (Householder, chunked; level 0 forms A1_low on the fly
    // and the chunk products M_c = Q_chunk^H V_chunk)
    ZFuse fz;
    if (k0 > 0) {
        fz.V = V + k0 * ldv;
        fz.ldv = ldv;
        fz.k0 = ik0;
        fz.K0P = P.K0P;
        fz.Zp = P.Zp;
        fz.Nc = P.Nc;
    }
    std::vector<ZLevel> Ls;
    if ((rc = ztsqr(P.ts, X0, ldx0, Q + k0 * ldq, ldq, R, ldr, st, k0 > 0 ? &fz : nullptr, &Ls, k0 == 0))) return rc;
    if (k0 > 0) {
        // G = W^H [0; Q_] = -V_low^H Q_ = -sum_c M_c^H G_c ;  N = T^{-1} G.
        // The k x k recurrence of the level-0 formation needs neither: it
        // runs on the side stream meanwhile.
        const int KP = P.ts.KP, K0P = P.K0P;
        Fork& f = fork_for_thread();
        if (!f.ok) return set_err(THO_E_HIP, "could not create the side stream");
        HIPCHK(hipEventRecord(f.ev0, st));
        HIPCHK(hipStreamWaitEvent(f.side, f.ev0, 0));
        PROF("zkchain_l0", f.side, launch_zkchain(KP, Ls[0], P.Cfin, f.side));
        HIPCHK(hipEventRecord(f.ev1, f.side));
        PROF("zchunk_prod", st, launch_zchunk_prod(Ls[0].nchunk, ik0, ik, KP, K0P, P.Nc, Ls[0].Gin, Ls[0].ldg,
                                                   Ls[0].gstride, P.prod, st));
        PROF("reduce_parts", st, launch_reduce_parts(Ls[0].nchunk, (int64_t)2 * K0P * KP, (const double*)P.prod,
                                                     (double*)P.Gsum, st));
        PROF("zsmall_ew", st, launch_zsmall_ew(ik0, ik, -1.0, P.Gsum, KP, 0, 0.0, nullptr, 0, 0, 0.0, 0, P.N, k, st));
        PROF("ztrsm", st, launch_ztrsm(ik0, ik, P.Tm, k0, 0, P.N, k, st));
        // level 0 of the formation with Q_low = Q_ + V_low N in the same pass
        PROF("zpermute", st, launch_zpermute_b(K0P, KP, ik0, ik, P.N, k, P.Np, st));
        HIPCHK(hipStreamWaitEvent(st, f.ev1, 0));
        PROF("zrows_l0", st, launch_zrows0(KP, K0P, Ls[0], P.Cfin, V + k0 * ldv, ldv, ik0, P.Np, st));
        // Q_top = -(P - V_top) N
        PROF("zgemm", st, launch_zgemm(ik0, ik, ik0, -1, 0, P.Pm, k0, 0, P.N, k, 0, 0, 0, nullptr, 0, Q, ldq, st));
        PROF("zgemm", st, launch_zgemm(ik0, ik, ik0, 1, 0, V, ldv, 0, P.N, k, 0, 1, 0, Q, ldq, Q, ldq, st));
    }
    return 0;
}

// ---- complex BCGS (same rounds/projections as the real tho_bcgs)
struct ZBcgsPlan {
    ZTsqrPlan ts;
    ZXty xc;
    ZRows rc;
    dcplx *C, *Sr, *Rr, *Rtmp;
    size_t bytes;
};

static void make_zbcgs_plan(int64_t n, int64_t k0, int64_t k, void* ws, ZBcgsPlan& P) {
    Carve cv(ws);
    ztsqr_plan(n, (int)k, cv, P.ts);
    P.C = P.Sr = nullptr;
    if (k0 > 0) {
        zxty_plan(n, (int)k0, (int)k, cv, P.xc);
        zrows_plan((int)k0, (int)k, cv, P.rc);
        P.C = ztake(cv, (size_t)k0 * k);
        P.Sr = ztake(cv, (size_t)k0 * k);
    }
    P.Rr = ztake(cv, (size_t)k * k);
    P.Rtmp = ztake(cv, (size_t)k * k);
    P.bytes = cv.bytes();
}

size_t zbcgs_bytes(int64_t n, int64_t k0, int64_t k) {
    if (k == 0) return 0;
    ZBcgsPlan P;
    make_zbcgs_plan(n, k0, k, nullptr, P);
    return P.bytes;
}

int run_zbcgs(int64_t n, int64_t k0, int64_t k, const dcplx* V, int64_t ldv, const dcplx* A, int64_t lda, dcplx* Q,
              int64_t ldq, dcplx* R, int64_t ldr, dcplx* S, int64_t lds, int proj, int rounds, void* ws,
              hipStream_t st) {
    int rc = 0;
    ZBcgsPlan P;
    make_zbcgs_plan(n, k0, k, ws, P);
    const int ik = (int)k, ik0 = (int)k0;
    const dcplx* X = A;
    int64_t ldx = lda;
    for (int r = 0; r < rounds; r++) {
        if (k0 > 0) {
            for (int p = 0; p < proj; p++) {
                if ((rc = zxty(P.xc, n, V, ldv, ik0, X, ldx, ik, 1.0, P.C, k, st))) return rc;
                if ((rc = zrows(P.rc, n, X, ldx, Q, ldq, V, ldv, ik0, P.C, k, ik, -1.0, st))) return rc;
                X = Q;
                ldx = ldq;
                // S_r (+)= C on the interleaved real view (k0 x 2k)
                PROF("small_ew", st, launch_small_ew(ik0, 2 * ik, p == 0 ? 0.0 : 1.0, p == 0 ? nullptr : (double*)P.Sr,
                                                     2 * k, 0, 1.0, (const double*)P.C, 2 * k, 0, 0.0, 0,
                                                     (double*)P.Sr, 2 * k, st));
            }
        }
        if ((rc = ztsqr(P.ts, X, ldx, Q, ldq, P.Rr, k, st))) return rc;
        X = Q;
        ldx = ldq;
        if (r == 0) {
            if (k0 > 0)
                PROF("zgemm", st, launch_zgemm(ik0, ik, 0, 0, 0, nullptr, 0, 0, nullptr, 0, 0, 1, 0, P.Sr, k, S, lds,
                                               st));
            PROF("zgemm", st, launch_zgemm(ik, ik, 0, 0, 0, nullptr, 0, 0, nullptr, 0, 0, 1, 0, P.Rr, k, R, ldr, st));
        } else {
            if (k0 > 0)
                PROF("zgemm", st, launch_zgemm(ik0, ik, ik, 1, 0, P.Sr, k, 0, R, ldr, 0, 1, 0, S, lds, S, lds, st));
            PROF("zgemm", st, launch_zgemm(ik, ik, ik, 1, 0, P.Rr, k, 0, R, ldr, 0, 0, 0, nullptr, 0, P.Rtmp, k, st));
            PROF("zgemm", st, launch_zgemm(ik, ik, 0, 0, 0, nullptr, 0, 0, nullptr, 0, 0, 1, 0, P.Rtmp, k, R, ldr, st));
        }
    }
    return 0;
}

// ---- complex full Householder QR of [V, A]: Algorithm 4 over 32-column panels
struct ZHhqrPlan {
    dcplx *Qv, *Rtmp, *Stmp;
    void* sub;
    size_t bytes;
};

static void make_zhhqr_plan(int64_t n, int64_t k0, int64_t k, void* ws, ZHhqrPlan& H) {
    Carve cv(ws);
    H.Qv = ztake(cv, (size_t)n * std::max<int64_t>(k0, 1));
    H.Rtmp = ztake(cv, 32 * 32);
    H.Stmp = ztake(cv, (size_t)std::max<int64_t>(k0, 1) * 32);
    size_t sub = ztwo_stage_bytes(n, k0, k);
    for (int64_t c = 0; c < k0; c += 32) sub = std::max(sub, ztwo_stage_bytes(n, c, std::min<int64_t>(32, k0 - c)));
    H.sub = cv.take(sub / sizeof(double) + 1);
    H.bytes = cv.bytes();
}

size_t zhhqr_bytes(int64_t n, int64_t k0, int64_t k) {
    if (k == 0) return 0;
    ZHhqrPlan H;
    make_zhhqr_plan(n, k0, k, nullptr, H);
    return H.bytes;
}

int run_zhhqr(int64_t n, int64_t k0, int64_t k, const dcplx* V, int64_t ldv, const dcplx* A, int64_t lda, dcplx* Q,
              int64_t ldq, dcplx* R, int64_t ldr, dcplx* S, int64_t lds, void* ws, hipStream_t st) {
    ZHhqrPlan H;
    make_zhhqr_plan(n, k0, k, ws, H);
    for (int64_t c = 0; c < k0; c += 32) {
        const int64_t w = std::min<int64_t>(32, k0 - c);
        int rc = run_ztwo_stage(n, c, w, H.Qv, k0, V + c, ldv, H.Qv + c, k0, H.Rtmp, 32, H.Stmp, 32, H.sub, st);
        if (rc) return rc;
    }
    return run_ztwo_stage(n, k0, k, H.Qv, k0, A, lda, Q, ldq, R, ldr, S, lds, H.sub, st);
}

}  // namespace tho

// ---- adjoint of (V, A) -> (Q, R, S) for complex128 (second choice of P).
// The steps of the real adjoint (tho_backward.cpp) with conjugate
// transposes; gradients follow dl = Re<V_bar, dV> + Re<A_bar, dA>,
// <X, Y> = sum conj(X) Y, for l = Re<G_Q, Q> + Re<G_R, R> + Re<G_S, S>.  The
// thin-QR adjoint of X = Q R (real positive diag R) is
//   X_bar = (Q_bar + Q copyltu(M)) R^{-H},  M = R R_bar^H - Q_bar^H Q,
// copyltu(M) = tril(M, -1) + tril(M, -1)^H + Re(diag M).
namespace {

// Out (nrows x q) = X + sum_t sign_t Y_t B_t, complex, one row-streaming pass.
struct ZRowsN {
    static constexpr int MAXT = 3;
    double *exp[MAXT], *pk[MAXT];
};
struct ZTerm {
    const dcplx* Y;
    int64_t ldy;
    int p;
    const dcplx* B;
    int64_t ldb;
    double sign;
};

void zrowsn_plan(int pmax, int q, Carve& cv, ZRowsN& Z) {
    for (int t = 0; t < ZRowsN::MAXT; t++) {
        Z.exp[t] = cv.take((size_t)4 * std::max(pmax, 1) * std::max(q, 1));
        Z.pk[t] = cv.take((size_t)k0p_of(2 * pmax) * rows_gemm_qp(2 * q) + 64);
    }
}

int zrowsn(const ZRowsN& Z, int64_t nrows, const dcplx* X, int64_t ldx, dcplx* Out, int64_t ldo, int q,
           std::initializer_list<ZTerm> terms, hipStream_t st) {
    RowsGemm g{};
    g.nrows = nrows;
    g.X = (const double*)X;
    g.ldx = 2 * ldx;
    g.Out = (double*)Out;
    g.ldo = 2 * ldo;
    g.q = 2 * q;
    g.nterm = 0;
    const int qp = rows_gemm_qp(2 * q);
    for (const ZTerm& t : terms) {
        const int i = g.nterm;
        const int kpad = k0p_of(2 * t.p);
        PROF("zexpand", st, launch_zexpand(t.p, q, t.B, t.ldb, t.sign, Z.exp[i], st));
        PROF("pack_b", st, launch_pack_b(2 * t.p, 2 * q, Z.exp[i], 2 * q, 0, 1.0, kpad, qp, Z.pk[i], st));
        g.t[g.nterm++] = {(const double*)t.Y, 2 * t.ldy, 2 * t.p, kpad, Z.pk[i]};
    }
    PROF("rows_gemm", st, launch_rows_gemm(g, st));
    return 0;
}

struct ZBwdPlan {
    ZXty xA, xQ, xG, xA1, xM;
    ZRowsN rr;
    dcplx *Pm, *Tm, *CA, *CQ, *CG, *CA1, *Z, *N, *Gb, *Yb, *A1t;
    dcplx *Qu, *Qub;
    dcplx *MQ, *gRu, *Mk, *CL, *RH, *RiH, *CM;
    dcplx *Tb, *Pb, *TmI, *TbL, *M1, *CL1, *B1m, *Li;
    size_t bytes;
};

void make_zbwd_plan(int64_t n, int64_t k0, int64_t k, void* ws, ZBwdPlan& P) {
    Carve cv(ws);
    const int ik = (int)k, ik0 = (int)k0;
    const size_t kk = (size_t)k * k, k0k = (size_t)std::max<int64_t>(k0, 1) * k,
                 k00 = (size_t)std::max<int64_t>(k0, 1) * std::max<int64_t>(k0, 1);
    zxty_plan(n - k0, ik, ik, cv, P.xM);
    zrowsn_plan(std::max(ik0, ik), std::max(ik0, ik), cv, P.rr);
    for (dcplx** p : {&P.MQ, &P.gRu, &P.Mk, &P.CL, &P.RH, &P.RiH, &P.CM}) *p = ztake(cv, kk);
    P.Pm = P.Tm = P.CA = P.CQ = P.CG = P.CA1 = P.Z = P.N = P.Gb = P.Yb = P.A1t = P.Qu = P.Qub = nullptr;
    P.Tb = P.Pb = P.TmI = P.TbL = P.M1 = P.CL1 = P.B1m = P.Li = nullptr;
    if (k0 > 0) {
        zxty_plan(n, ik0, ik, cv, P.xA);
        zxty_plan(n, ik0, ik, cv, P.xQ);
        zxty_plan(n, ik0, ik, cv, P.xG);
        zxty_plan(n, ik0, ik, cv, P.xA1);
        for (dcplx** p : {&P.CA, &P.CQ, &P.CG, &P.CA1, &P.Z, &P.N, &P.Gb, &P.Yb, &P.A1t}) *p = ztake(cv, k0k);
        for (dcplx** p : {&P.Pm, &P.Tm, &P.Tb, &P.Pb, &P.TmI, &P.TbL, &P.M1, &P.CL1, &P.B1m, &P.Li})
            *p = ztake(cv, k00);
        P.Qu = ztake(cv, (size_t)(n - k0) * k);
        P.Qub = ztake(cv, (size_t)(n - k0) * k);
    }
    P.bytes = cv.bytes();
}

}  // namespace

namespace tho {

size_t ztwo_stage_backward_bytes(int64_t n, int64_t k0, int64_t k) {
    if (k == 0) return 0;
    ZBwdPlan P;
    make_zbwd_plan(n, k0, k, nullptr, P);
    return P.bytes;
}

int run_ztwo_stage_backward(int64_t n, int64_t k0, int64_t k, const dcplx* V, int64_t ldv, const dcplx* A,
                            int64_t lda, const dcplx* Q, int64_t ldq, const dcplx* R, int64_t ldr, const dcplx* gQ,
                            int64_t ldgq, const dcplx* gR, int64_t ldgr, const dcplx* gS, int64_t ldgs, dcplx* dV,
                            int64_t lddv, dcplx* dA, int64_t ldda, void* ws, hipStream_t st) {
    int rc = 0;
    ZBwdPlan P;
    make_zbwd_plan(n, k0, k, ws, P);
    const int ik = (int)k, ik0 = (int)k0;
    const int64_t m = n - k0;
    const dcplx *Qu = Q + k0 * ldq, *Qub = gQ + k0 * ldgq;
    int64_t ldqu = ldq, ldqub = ldgq;
    if (k0 > 0) {
        // P, T again (side stream) beside the reductions V^H A, V^H Q, V^H G_Q
        Fork& f = fork_for_thread();
        if (!f.ok) return set_err(THO_E_HIP, "could not create the side stream");
        HIPCHK(hipEventRecord(f.ev0, st));
        HIPCHK(hipStreamWaitEvent(f.side, f.ev0, 0));
        PROF("zqr_top", f.side, launch_zqr_top(ik0, V, ldv, P.Pm, P.Tm, f.side));
        HIPCHK(hipEventRecord(f.ev1, f.side));
        if ((rc = zxty(P.xA, n, V, ldv, ik0, A, lda, ik, 1.0, P.CA, k, st))) return rc;
        if ((rc = zxty(P.xQ, n, V, ldv, ik0, Q, ldq, ik, 1.0, P.CQ, k, st))) return rc;
        if ((rc = zxty(P.xG, n, V, ldv, ik0, gQ, ldgq, ik, 1.0, P.CG, k, st))) return rc;
        HIPCHK(hipStreamWaitEvent(st, f.ev1, 0));
        // Z = T^{-H} (P^H A_top - V^H A)
        PROF("zgemm", st, launch_zgemm(ik0, ik, ik0, 1, 0, P.Pm, k0, 2, A, lda, 0, -1, 0, P.CA, k, P.Z, k, st));
        PROF("ztrsm", st, launch_ztrsm(ik0, ik, P.Tm, k0, 2, P.Z, k, st));
        // N = -T^{-H} W^H Q  (W^H W = T + T^H for orthonormal V)
        PROF("zgemm", st, launch_zgemm(ik0, ik, ik0, -1, 0, P.Pm, k0, 2, Q, ldq, 0, 1, 0, P.CQ, k, P.N, k, st));
        PROF("ztrsm", st, launch_ztrsm(ik0, ik, P.Tm, k0, 2, P.N, k, st));
        // G_bar = T^{-H} N_bar, N_bar = -W^H Q_bar
        PROF("zgemm", st, launch_zgemm(ik0, ik, ik0, -1, 0, P.Pm, k0, 2, gQ, ldgq, 0, 1, 0, P.CG, k, P.Gb, k, st));
        PROF("ztrsm", st, launch_ztrsm(ik0, ik, P.Tm, k0, 2, P.Gb, k, st));
        // Q_ = Q_low - V_low N ;  Q__bar = Q_bar_low - V_low G_bar
        if ((rc = zrowsn(P.rr, m, Q + k0 * ldq, ldq, P.Qu, k, ik, {{V + k0 * ldv, ldv, ik0, P.N, k, -1.0}}, st)))
            return rc;
        if ((rc = zrowsn(P.rr, m, gQ + k0 * ldgq, ldgq, P.Qub, k, ik, {{V + k0 * ldv, ldv, ik0, P.Gb, k, -1.0}}, st)))
            return rc;
        Qu = P.Qu;
        Qub = P.Qub;
        ldqu = ldqub = k;
    }
    // (QR) adjoint: A1_bar_low = (Q__bar + Q_ copyltu(M)) R^{-H},
    // M = R triu(R_bar)^H - Q__bar^H Q_
    if ((rc = zxty(P.xM, m, Qub, ldqub, ik, Qu, ldqu, ik, 1.0, P.MQ, k, st))) return rc;
    PROF("zsmall_ew", st, launch_zsmall_ew(ik, ik, 1.0, gR, ldgr, 0, 0.0, nullptr, 0, 0, 0.0, 2, P.gRu, k, st));
    PROF("zgemm", st, launch_zgemm(ik, ik, ik, 1, 0, R, ldr, 0, P.gRu, k, 2, -1, 0, P.MQ, k, P.Mk, k, st));
    PROF("zsmall_ew", st, launch_zsmall_ew(ik, ik, 1.0, P.Mk, k, 0, 0.0, nullptr, 0, 0, 0.0, 3, P.CL, k, st));
    // R^{-H}: solve R^H X = I with R^H stored lower
    PROF("zsmall_ew", st, launch_zsmall_ew(ik, ik, 1.0, R, ldr, 2, 0.0, nullptr, 0, 0, 0.0, 1, P.RH, k, st));
    PROF("zsmall_ew", st, launch_zsmall_ew(ik, ik, 0.0, nullptr, 0, 0, 0.0, nullptr, 0, 0, 1.0, 0, P.RiH, k, st));
    PROF("ztrsm", st, launch_ztrsm(ik, ik, P.RH, k, 0, P.RiH, k, st));
    PROF("zgemm", st, launch_zgemm(ik, ik, ik, 1, 0, P.CL, k, 0, P.RiH, k, 0, 0, 0, nullptr, 0, P.CM, k, st));
    if ((rc = zrowsn(P.rr, m, nullptr, 0, dA + k0 * ldda, ldda, ik,
                     {{Qub, ldqub, ik, P.RiH, k, 1.0}, {Qu, ldqu, ik, P.CM, k, 1.0}}, st)))
        return rc;
    if (k0 == 0) return 0;

    // (S) adjoint: A1_bar_top = P S_bar
    if (gS)
        PROF("zgemm", st, launch_zgemm(ik0, ik, ik0, 1, 0, P.Pm, k0, 0, gS, ldgs, 0, 0, 0, nullptr, 0, dA, ldda, st));
    else
        PROF("zsmall_ew", st, launch_zsmall_ew(ik0, ik, 0.0, nullptr, 0, 0, 0.0, nullptr, 0, 0, 0.0, 0, dA, ldda, st));
    // (A) adjoint: Y_bar = T^{-1} Z_bar, Z_bar = -W^H A1_bar = V^H A1_bar - P^H A1_bar_top
    if ((rc = zxty(P.xA1, n, V, ldv, ik0, dA, ldda, ik, 1.0, P.CA1, k, st))) return rc;
    PROF("zgemm", st, launch_zgemm(ik0, ik, ik0, -1, 0, P.Pm, k0, 2, dA, ldda, 0, 1, 0, P.CA1, k, P.Yb, k, st));
    PROF("ztrsm", st, launch_ztrsm(ik0, ik, P.Tm, k0, 0, P.Yb, k, st));
    // T_bar = -G_bar N^H - Z Y_bar^H
    PROF("zgemm", st, launch_zgemm(ik0, ik0, ik, -1, 0, P.Gb, k, 0, P.N, k, 2, 0, 0, nullptr, 0, P.Tb, k0, st));
    PROF("zgemm", st, launch_zgemm(ik0, ik0, ik, -1, 0, P.Z, k, 0, P.Yb, k, 2, 1, 0, P.Tb, k0, P.Tb, k0, st));
    // V_bar = -W_bar = Q_bar N^H - [0; Q_] G_bar^H + A1_bar Z^H - A Y_bar^H
    // (B operands are the conjugate transposes, k x k0)
    PROF("zsmall_ew", st, launch_zsmall_ew(ik, ik0, 1.0, P.N, k, 2, 0.0, nullptr, 0, 0, 0.0, 0, P.CA, k0, st));
    PROF("zsmall_ew", st, launch_zsmall_ew(ik, ik0, 1.0, P.Z, k, 2, 0.0, nullptr, 0, 0, 0.0, 0, P.CQ, k0, st));
    PROF("zsmall_ew", st, launch_zsmall_ew(ik, ik0, 1.0, P.Yb, k, 2, 0.0, nullptr, 0, 0, 0.0, 0, P.CG, k0, st));
    if ((rc = zrowsn(P.rr, n, nullptr, 0, dV, lddv, ik0,
                     {{gQ, ldgq, ik, P.CA, k0, 1.0}, {dA, ldda, ik, P.CQ, k0, 1.0}, {A, lda, ik, P.CG, k0, -1.0}},
                     st)))
        return rc;
    PROF("zsmall_ew", st, launch_zsmall_ew(ik, ik0, 1.0, P.Gb, k, 2, 0.0, nullptr, 0, 0, 0.0, 0, P.CA, k0, st));
    if ((rc = zrowsn(P.rr, m, dV + k0 * lddv, lddv, dV + k0 * lddv, lddv, ik0, {{P.Qu, k, ik, P.CA, k0, -1.0}}, st)))
        return rc;
    // P_bar = A1_top S_bar^H + W_bar_top,  A1_top = A_top - (P - V_top) Z
    PROF("zgemm", st, launch_zgemm(ik0, ik, ik0, -1, 0, P.Pm, k0, 0, P.Z, k, 0, 1, 0, A, lda, P.A1t, k, st));
    PROF("zgemm", st, launch_zgemm(ik0, ik, ik0, 1, 0, V, ldv, 0, P.Z, k, 0, 1, 0, P.A1t, k, P.A1t, k, st));
    if (gS)
        PROF("zgemm", st, launch_zgemm(ik0, ik0, ik, 1, 0, P.A1t, k, 0, gS, ldgs, 2, -1, 0, dV, lddv, P.Pb, k0, st));
    else
        PROF("zsmall_ew", st, launch_zsmall_ew(ik0, ik0, -1.0, dV, lddv, 0, 0.0, nullptr, 0, 0, 0.0, 0, P.Pb, k0, st));
    // A_bar = A1_bar + W Y_bar: bottom rows - V_low Y_bar, top rows + (P - V_top) Y_bar
    if ((rc = zrowsn(P.rr, m, dA + k0 * ldda, ldda, dA + k0 * ldda, ldda, ik, {{V + k0 * ldv, ldv, ik0, P.Yb, k, -1.0}},
                     st)))
        return rc;
    PROF("zgemm", st, launch_zgemm(ik0, ik, ik0, 1, 0, P.Pm, k0, 0, P.Yb, k, 0, 1, 0, dA, ldda, dA, ldda, st));
    PROF("zgemm", st, launch_zgemm(ik0, ik, ik0, -1, 0, V, ldv, 0, P.Yb, k, 0, 1, 0, dA, ldda, dA, ldda, st));
    // (P, T) adjoint: V_top = Q1 R1, Q1 = -P, R1 = (T - I)^H, Q1_bar = -P_bar,
    // R1_bar = tril(T_bar)^H:  M1 = (T - I)^H tril(T_bar) - P_bar^H P,
    // V_bar_top += (-P_bar - P copyltu(M1)) (T - I)^{-1}
    PROF("zsmall_ew", st, launch_zsmall_ew(ik0, ik0, 1.0, P.Tm, k0, 0, 0.0, nullptr, 0, 0, -1.0, 1, P.TmI, k0, st));
    PROF("zsmall_ew", st, launch_zsmall_ew(ik0, ik0, 1.0, P.Tb, k0, 0, 0.0, nullptr, 0, 0, 0.0, 1, P.TbL, k0, st));
    PROF("zgemm", st, launch_zgemm(ik0, ik0, ik0, 1, 0, P.TmI, k0, 2, P.TbL, k0, 0, 0, 0, nullptr, 0, P.M1, k0, st));
    PROF("zgemm", st, launch_zgemm(ik0, ik0, ik0, -1, 0, P.Pb, k0, 2, P.Pm, k0, 0, 1, 0, P.M1, k0, P.M1, k0, st));
    PROF("zsmall_ew", st, launch_zsmall_ew(ik0, ik0, 1.0, P.M1, k0, 0, 0.0, nullptr, 0, 0, 0.0, 3, P.CL1, k0, st));
    PROF("zgemm", st, launch_zgemm(ik0, ik0, ik0, -1, 0, P.Pm, k0, 0, P.CL1, k0, 0, -1, 0, P.Pb, k0, P.B1m, k0, st));
    PROF("zsmall_ew", st, launch_zsmall_ew(ik0, ik0, 0.0, nullptr, 0, 0, 0.0, nullptr, 0, 0, 1.0, 0, P.Li, k0, st));
    PROF("ztrsm", st, launch_ztrsm(ik0, ik0, P.TmI, k0, 0, P.Li, k0, st));
    PROF("zgemm", st, launch_zgemm(ik0, ik0, ik0, 1, 0, P.B1m, k0, 0, P.Li, k0, 0, 1, 0, dV, lddv, dV, lddv, st));
    return 0;
}

}  // namespace tho
