// Block Householder-QR of column blocks A = [A_1, ..., A_p] (Algorithm 4,
// §6.1): each block is orthogonalized against the basis of the blocks before
// it by a generalized Householder transformation and its bottom rows are
// Householder-QR factored, so the basis may grow past the width one
// two-stage step takes (any total width; every block at most 64 columns).
//
// The H of block i is built from V = [Q_1, ..., Q_{i-1}] with the block
// diagonal P = diag(P_1, ..., P_{i-1}), P_j from the top block of the
// block's own bottom basis Qu_j (the Q_ of its QR, rows o_j.. with
// o_j = k_1 + ... + k_{j-1}).  With that P, H factors as
//     H = H_1' H_2' ... H_{i-1}',
// H_j' the generalized Householder transformation of Algorithm 1 for Qu_j,
// acting on rows o_j..n (H_1'^* Q_2 = [0; Qu_2], and so on).  So block i
// runs, with kernels of the two-stage path:
//     X = A_i;  X[o_j:] <- H_j'^* X[o_j:]  (j = 1 .. i-1)
//     S_i's block j = P_j^* X[o_j : o_j + k_j]
//     X[o_i:] = Qu_i R_i (Householder QR);  P_i, T_i from Qu_i's top block
//     Q_i = [0; Qu_i];  Q_i[o_j:] <- H_j' Q_i[o_j:]  (j = i-1 .. 1)
// In exact arithmetic Q and R do not depend on the choice of P.
#include <algorithm>
#include <numeric>
#include <vector>

#include "tho_host.h"

using namespace tho;

namespace {

// Workspace of a basis of up to kmax columns over n rows.
struct BlockPlan {
    int64_t n = 0, kmax = 0;
    XtyPlan xp;
    double *Qu = nullptr;                        // n x kmax, ld kmax: bottom bases Qu_j
    double *Pall = nullptr, *Tall = nullptr, *F2all = nullptr;  // block j at offset 64 c_j, ld k_j
    double *pws = nullptr;                       // polar workspace (k <= 64)
    double *part = nullptr, *C = nullptr, *Z = nullptr, *Zpk = nullptr;
    void* qrws = nullptr;                        // plain Householder QR of a block
    size_t bytes = 0;
};

void make_block_plan(int64_t n, int64_t kmax, void* ws, BlockPlan& B) {
    Carve cv(ws);
    B.n = n;
    B.kmax = kmax;
    B.xp = xty_plan(n);
    B.Qu = cv.take((size_t)n * kmax);
    B.Pall = cv.take((size_t)kmax * 64);
    B.Tall = cv.take((size_t)kmax * 64);
    B.F2all = cv.take((size_t)kmax * 64);
    B.pws = cv.take(pchoice_ws_doubles(64));
    B.part = cv.take((size_t)B.xp.nblk * 64 * 64);
    B.C = cv.take(64 * 64);
    B.Z = cv.take(64 * 64);
    B.Zpk = cv.take(64 * 64);
    B.qrws = cv.take(plain_qr_bytes(n, 64) / sizeof(double) + 1);
    B.bytes = cv.bytes();
}

RowsGemm rows_op(int64_t nrows, const double* X, int64_t ldx, double* Out, int64_t ldo, int q) {
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

// X[o_j:] <- H_j'^* X[o_j:] (adjoint) or H_j' X[o_j:]:
//   Y = W^T X = P_j^T X_top - Qu_j^T X,  Z = T_j^{-T} Y (or T_j^{-1} Y),
//   X <- X - W Z = X + Qu_j Z  and  X_top <- X_top - P_j Z.
// X: m = n - o_j rows starting at row o_j, kx columns (ld ldx).
int apply_gh(bool adjoint, int pchoice, const BlockPlan& B, int64_t m, int kj, const double* Vj, const double* Pj,
             const double* Tj, const double* F2j, double* X, int64_t ldx, int kx, hipStream_t st) {
    const int KPX = kp_of(kx);
    int rc = xty(B.xp, m, Vj, B.kmax, kj, X, ldx, kx, B.part, B.C, st, "xty_partial");
    if (rc) return rc;
    PROF("small_gemm", st, launch_small_gemm(kj, kx, kj, 1.0, Pj, kj, 1, X, ldx, 0, -1.0, B.C, KPX, B.Z, KPX, st));
    rc = adjoint ? solve_tt(pchoice, kj, kx, Tj, F2j, B.Z, KPX, st) : solve_t(pchoice, kj, kx, Tj, F2j, B.Z, KPX, st);
    if (rc) return rc;
    const int kpad = k0p_of(kj), qp = rows_gemm_qp(kx);
    PROF("pack_b", st, launch_pack_b(kj, kx, B.Z, KPX, 0, 1.0, kpad, qp, B.Zpk, st));
    RowsGemm g = rows_op(m, X, ldx, X, ldx, kx);
    g.t[g.nterm++] = {Vj, B.kmax, kj, kpad, B.Zpk};
    PROF("rows_gemm", st, launch_rows_gemm(g, st));
    PROF("small_gemm", st, launch_small_gemm(kj, kx, kj, -1.0, Pj, kj, 0, B.Z, KPX, 0, 1.0, X, ldx, X, ldx, st));
    return 0;
}

// Block i (0-based) of the basis; blocks 0..i-1 are already in Q and in the
// workspace.  Writes Q[:, c_i : c_i + k_i] and R[0 : c_i + k_i, c_i : c_i + k_i].
int block_step(int pchoice, const BlockPlan& B, int i, const int64_t* kb, const double* Ai, int64_t lda, double* Q,
               int64_t ldq, double* R, int64_t ldr, hipStream_t st) {
    const int64_t n = B.n;
    std::vector<int64_t> c(i + 1, 0);
    for (int j = 1; j <= i; j++) c[j] = c[j - 1] + kb[j - 1];
    const int ki = (int)kb[i];
    const int64_t ci = c[i];
    double* X = Q + ci;
    int rc = 0;
    // X = A_i
    {
        RowsGemm g = rows_op(n, Ai, lda, X, ldq, ki);
        PROF("rows_gemm", st, launch_rows_gemm(g, st));
    }
    // X <- H_{i-1}'^* ... H_1'^* X, and the blocks of S_i
    for (int j = 0; j < i; j++) {
        const int kj = (int)kb[j];
        const int64_t oj = c[j];
        const double* Vj = B.Qu + oj * B.kmax + oj;
        const double* Pj = B.Pall + 64 * oj;
        if ((rc = apply_gh(true, pchoice, B, n - oj, kj, Vj, Pj, B.Tall + 64 * oj, B.F2all + 64 * oj, X + oj * ldq,
                           ldq, ki, st)))
            return rc;
        PROF("small_gemm", st, launch_small_gemm(kj, ki, kj, 1.0, Pj, kj, 1, X + oj * ldq, ldq, 0, 0.0, nullptr, 0,
                                                 R + oj * ldr + ci, ldr, st));
    }
    // X[o_i:] = Qu_i R_i, then P_i, T_i from the top block of Qu_i
    double* Qui = B.Qu + ci * B.kmax + ci;
    if ((rc = run_plain_qr(n - ci, ki, X + ci * ldq, ldq, Qui, B.kmax, R + ci * ldr + ci, ldr, B.qrws, st))) return rc;
    if ((rc = p_and_t(pchoice, ki, Qui, B.kmax, B.Pall + 64 * ci, B.Tall + 64 * ci, B.F2all + 64 * ci, B.pws, st)))
        return rc;
    // Q_i = H_1' ... H_{i-1}' [0; Qu_i]
    if (ci > 0)
        PROF("small_ew", st, launch_small_ew((int)ci, ki, 0.0, nullptr, 0, 0, 0.0, nullptr, 0, 0, 0.0, 0, X, ldq, st));
    {
        RowsGemm g = rows_op(n - ci, Qui, B.kmax, X + ci * ldq, ldq, ki);
        PROF("rows_gemm", st, launch_rows_gemm(g, st));
    }
    for (int j = i - 1; j >= 0; j--) {
        const int kj = (int)kb[j];
        const int64_t oj = c[j];
        if ((rc = apply_gh(false, pchoice, B, n - oj, kj, B.Qu + oj * B.kmax + oj, B.Pall + 64 * oj,
                           B.Tall + 64 * oj, B.F2all + 64 * oj, X + oj * ldq, ldq, ki, st)))
            return rc;
    }
    return 0;
}

int check_blocks(int32_t dtype, int64_t n, int32_t nb, const int64_t* kb, int64_t* ktot) {
    if (dtype != THO_F64) return set_err(THO_E_UNSUPPORTED, "block Householder-QR is implemented for THO_F64 only");
    if (n < 0) return set_err(-2, "n must be >= 0");
    if (nb < 0) return set_err(-3, "number of blocks must be >= 0");
    if (nb > 0 && !kb) return set_err(-4, "block widths are NULL");
    int64_t t = 0;
    for (int i = 0; i < nb; i++) {
        if (kb[i] < 1 || kb[i] > THO_MAX_K) return set_err(-4, "every block width must be in [1, THO_MAX_K]");
        t += kb[i];
    }
    if (t > n) return set_err(-2, "need n >= total number of columns");
    *ktot = t;
    return 0;
}

}  // namespace

extern "C" {

int tho_block_householder_workspace(int32_t dtype, int64_t n, int64_t kmax, const tho_opts_t* opts, size_t* bytes) {
    if (dtype != THO_F64) return set_err(THO_E_UNSUPPORTED, "block Householder-QR is implemented for THO_F64 only");
    if (n < 0) return set_err(-2, "n must be >= 0");
    if (kmax < 0 || kmax > n) return set_err(-3, "need 0 <= kmax <= n");
    if (!bytes) return set_err(-5, "bytes must not be NULL");
    (void)opts;
    if (kmax == 0) { *bytes = 0; return 0; }
    BlockPlan B;
    make_block_plan(n, kmax, nullptr, B);
    *bytes = B.bytes;
    return 0;
}

int tho_block_householder_step(int32_t dtype, int64_t n, int32_t i, const int64_t* kb, int64_t kmax, const void* Ai,
                               int64_t lda, void* Q, int64_t ldq, void* R, int64_t ldr, const tho_opts_t* opts,
                               void* ws, size_t ws_bytes, void* stream) {
    int64_t ktot = 0;
    int rc = check_blocks(dtype, n, i + 1, kb, &ktot);
    if (rc) return rc;
    if (i < 0) return set_err(-3, "block index must be >= 0");
    if (ktot > kmax || kmax > n) return set_err(-5, "need sum of widths <= kmax <= n");
    const int pchoice = opts ? opts->p_choice : THO_P_QR;
    if (opts && (opts->panel != THO_PANEL_F64 || opts->flags != 0)) return set_err(THO_E_UNSUPPORTED, "default panel, no flags");
    if (pchoice < THO_P_QR || pchoice > THO_P_POLAR) return set_err(-12, "unknown choice of P");
    const int64_t ki = kb[i];
    if (!Ai) return set_err(-6, "A_i is NULL");
    if (lda < ki) return set_err(-7, "lda < k_i");
    if (!Q) return set_err(-8, "Q is NULL");
    if (ldq < ktot) return set_err(-9, "ldq < sum of widths");
    if (!R) return set_err(-10, "R is NULL");
    if (ldr < ktot) return set_err(-11, "ldr < sum of widths");
    for (const void* p : {Ai, (const void*)Q, (const void*)R})
        if ((uintptr_t)p & 7) return set_err(-6, "matrices must be 8-byte aligned");
    const int64_t ci = ktot - ki;
    if (blocks_overlap(Q, n, ktot, ldq, Ai, n, ki, lda, 8)) return set_err(-8, "Q overlaps A_i");
    if (blocks_overlap(R, ktot, ktot, ldr, Ai, n, ki, lda, 8) || blocks_overlap(R, ktot, ktot, ldr, Q, n, ktot, ldq, 8))
        return set_err(-10, "R overlaps A_i or Q");
    (void)ci;
    if (!ws) return set_err(-13, "workspace is NULL");
    BlockPlan B;
    make_block_plan(n, kmax, nullptr, B);
    if (ws_bytes < B.bytes) return set_err(THO_E_WORKSPACE, "workspace too small");
    make_block_plan(n, kmax, ws, B);
    return block_step(pchoice, B, i, kb, (const double*)Ai, lda, (double*)Q, ldq, (double*)R, ldr,
                      (hipStream_t)stream);
}

int tho_block_householder(int32_t dtype, int64_t n, int32_t nblocks, const int64_t* kb, const void* A, int64_t lda,
                          void* Q, int64_t ldq, void* R, int64_t ldr, const tho_opts_t* opts, void* ws,
                          size_t ws_bytes, void* stream) {
    int64_t ktot = 0;
    int rc = check_blocks(dtype, n, nblocks, kb, &ktot);
    if (rc) return rc;
    if (ktot == 0) return 0;
    const int pchoice = opts ? opts->p_choice : THO_P_QR;
    if (opts && (opts->panel != THO_PANEL_F64 || opts->flags != 0)) return set_err(THO_E_UNSUPPORTED, "default panel, no flags");
    if (pchoice < THO_P_QR || pchoice > THO_P_POLAR) return set_err(-11, "unknown choice of P");
    if (!A) return set_err(-5, "A is NULL");
    if (lda < ktot) return set_err(-6, "lda < number of columns");
    if (!Q) return set_err(-7, "Q is NULL");
    if (ldq < ktot) return set_err(-8, "ldq < number of columns");
    if (!R) return set_err(-9, "R is NULL");
    if (ldr < ktot) return set_err(-10, "ldr < number of columns");
    for (const void* p : {A, (const void*)Q, (const void*)R})
        if ((uintptr_t)p & 7) return set_err(-5, "matrices must be 8-byte aligned");
    if (blocks_overlap(Q, n, ktot, ldq, A, n, ktot, lda, 8)) return set_err(-7, "Q overlaps A");
    if (blocks_overlap(R, ktot, ktot, ldr, A, n, ktot, lda, 8) || blocks_overlap(R, ktot, ktot, ldr, Q, n, ktot, ldq, 8))
        return set_err(-9, "R overlaps A or Q");
    if (!ws) return set_err(-12, "workspace is NULL");
    BlockPlan B;
    make_block_plan(n, ktot, nullptr, B);
    if (ws_bytes < B.bytes) return set_err(THO_E_WORKSPACE, "workspace too small");
    make_block_plan(n, ktot, ws, B);
    hipStream_t st = (hipStream_t)stream;
    double* Rd = (double*)R;
    // R is upper triangular: clear it first (each step writes the rows
    // 0 .. c_i + k_i - 1 of its block column)
    PROF("small_ew", st, launch_small_ew((int)ktot, (int)ktot, 0.0, nullptr, 0, 0, 0.0, nullptr, 0, 0, 0.0, 0, Rd, ldr,
                                         st));
    int64_t c = 0;
    for (int i = 0; i < nblocks; i++) {
        if ((rc = block_step(pchoice, B, i, kb, (const double*)A + c, lda, (double*)Q, ldq, Rd, ldr, st))) return rc;
        c += kb[i];
    }
    return 0;
}

}  // extern "C"
