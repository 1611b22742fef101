// Small dense kernels: split-n reductions of X^T Y (the V^*A products of
// Algorithm 1), their fixed-order finish, and the k0 x k0 / k0 x k work
// done by one workgroup (QR of the top block for the second choice of P,
// triangular solves with T, small products).
#include "tho_device.h"
#include "tho_internal.h"
#include "small_dev.h"

namespace tho {

// --------------------------------------------------------------------------
// part[blk] = X[r0:r1]^T Y[r0:r1] for the row range of block blk.
// X: nrows x p (ld ldx), Y: nrows x q (ld ldy), p <= 16*MT, q <= 16*NT.
// Four waves: WM wave groups split the MT row-tiles of the output, the
// remaining 4/WM groups split the rows and are summed through LDS.
// Every K-step consumes 4 rows; operands are read straight from HBM in the
// MFMA operand layouts (16 consecutive doubles of one row per lane group).
// Output: part[blk][16*MT][16*NT], row-major.
// --------------------------------------------------------------------------
template <int MT, int NT, int WM>
__global__ __launch_bounds__(256, 3) void k_xty_partial(
    int64_t nrows, const double* __restrict__ X, int64_t ldx, int p,
    const double* __restrict__ Y, int64_t ldy, int q, int64_t rows_per_blk,
    double* __restrict__ part) {
    constexpr int MTW = MT / WM;
    constexpr int WR = 4 / WM;
    constexpr int RED = (WR > 1) ? (WR - 1) * WM * MTW * NT * 64 : 1;
    __shared__ d4 red[RED];
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wm = w % WM, wr = w / WM;
    const int g = l >> 4, cl = l & 15;
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_blk;
    const int64_t r1 = (r0 + rows_per_blk < nrows) ? r0 + rows_per_blk : nrows;

    d4 acc[MTW][NT];
#pragma unroll
    for (int i = 0; i < MTW; i++)
#pragma unroll
        for (int j = 0; j < NT; j++) acc[i][j] = d4zero();

    int colx[MTW];
    bool okx[MTW];
#pragma unroll
    for (int i = 0; i < MTW; i++) {
        colx[i] = 16 * (wm * MTW + i) + cl;
        okx[i] = colx[i] < p;
    }
    int coly[NT];
    bool oky[NT];
#pragma unroll
    for (int j = 0; j < NT; j++) {
        coly[j] = 16 * j + cl;
        oky[j] = coly[j] < q;
    }
    // 16 rows (4 K-steps) per iteration of this wave; wave groups interleave
    constexpr int U = 4;
    for (int64_t rb = r0 + (int64_t)wr * 4 * U; rb < r1; rb += (int64_t)WR * 4 * U) {
        double xa[U][MTW], yb[U][NT];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int64_t row = rb + 4 * u + g;
            const bool rv = row < r1;
#pragma unroll
            for (int i = 0; i < MTW; i++)
                xa[u][i] = (rv && okx[i]) ? X[row * ldx + colx[i]] : 0.0;
#pragma unroll
            for (int j = 0; j < NT; j++)
                yb[u][j] = (rv && oky[j]) ? Y[row * ldy + coly[j]] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; u++)
#pragma unroll
            for (int i = 0; i < MTW; i++)
#pragma unroll
                for (int j = 0; j < NT; j++) acc[i][j] = mfma(xa[u][i], yb[u][j], acc[i][j]);
    }
    if (WR > 1) {
        if (wr > 0) {
#pragma unroll
            for (int i = 0; i < MTW; i++)
#pragma unroll
                for (int j = 0; j < NT; j++)
                    red[(((wr - 1) * WM + wm) * MTW * NT + i * NT + j) * 64 + l] = acc[i][j];
        }
        __syncthreads();
        if (wr == 0) {
            for (int r = 1; r < WR; r++)
#pragma unroll
                for (int i = 0; i < MTW; i++)
#pragma unroll
                    for (int j = 0; j < NT; j++)
                        acc[i][j] += red[(((r - 1) * WM + wm) * MTW * NT + i * NT + j) * 64 + l];
        }
    }
    if (wr == 0) {
        double* out = part + (int64_t)blockIdx.x * (16 * MT) * (16 * NT);
#pragma unroll
        for (int i = 0; i < MTW; i++)
#pragma unroll
            for (int j = 0; j < NT; j++)
#pragma unroll
                for (int v = 0; v < 4; v++) {
                    const int row = 16 * (wm * MTW + i) + drow(l, v);
                    out[row * (16 * NT) + 16 * j + cl] = acc[i][j][v];
                }
    }
}

// part[blk] = X[r0:r1]^T [Y0 Y1 Y2][r0:r1] for three matrices of q columns
// each (the adjoint's V^T [A, Q, G_Q]), read in one pass over X: output
// (16 MT) x (3 * 16 NB) row-major, the blocks of Y_i side by side.  Same
// structure as k_xty_partial with WM = MT wave groups over the row tiles.
template <int MT, int NB>
__global__ __launch_bounds__(256, 2) void k_xty3_partial(int64_t nrows, const double* __restrict__ X, int64_t ldx,
                                                         int p, const double* __restrict__ Y0, int64_t ld0,
                                                         const double* __restrict__ Y1, int64_t ld1,
                                                         const double* __restrict__ Y2, int64_t ld2, int q,
                                                         int64_t rows_per_blk, double* __restrict__ part) {
    constexpr int WM = (MT >= 4) ? 4 : MT;
    constexpr int MTW = MT / WM;
    constexpr int WR = 4 / WM;
    constexpr int NT = 3 * NB;
    constexpr int RED = (WR > 1) ? (WR - 1) * WM * MTW * NT * 64 : 1;
    __shared__ d4 red[RED];
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wm = w % WM, wr = w / WM;
    const int g = l >> 4, cl = l & 15;
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_blk;
    const int64_t r1 = (r0 + rows_per_blk < nrows) ? r0 + rows_per_blk : nrows;
    d4 acc[MTW][NT];
#pragma unroll
    for (int i = 0; i < MTW; i++)
#pragma unroll
        for (int j = 0; j < NT; j++) acc[i][j] = d4zero();
    int colx[MTW];
    bool okx[MTW];
#pragma unroll
    for (int i = 0; i < MTW; i++) {
        colx[i] = 16 * (wm * MTW + i) + cl;
        okx[i] = colx[i] < p;
    }
    constexpr int U = 2;
    for (int64_t rb = r0 + (int64_t)wr * 4 * U; rb < r1; rb += (int64_t)WR * 4 * U) {
        double xa[U][MTW], yb[U][NT];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int64_t row = rb + 4 * u + g;
            const bool rv = row < r1;
#pragma unroll
            for (int i = 0; i < MTW; i++) xa[u][i] = (rv && okx[i]) ? X[row * ldx + colx[i]] : 0.0;
#pragma unroll
            for (int j = 0; j < NB; j++) {
                const int cy = 16 * j + cl;
                const bool ok = rv && cy < q;
                yb[u][j] = ok ? Y0[row * ld0 + cy] : 0.0;
                yb[u][NB + j] = ok ? Y1[row * ld1 + cy] : 0.0;
                yb[u][2 * NB + j] = ok ? Y2[row * ld2 + cy] : 0.0;
            }
        }
#pragma unroll
        for (int u = 0; u < U; u++)
#pragma unroll
            for (int i = 0; i < MTW; i++)
#pragma unroll
                for (int j = 0; j < NT; j++) acc[i][j] = mfma(xa[u][i], yb[u][j], acc[i][j]);
    }
    if (WR > 1) {
        if (wr > 0) {
#pragma unroll
            for (int i = 0; i < MTW; i++)
#pragma unroll
                for (int j = 0; j < NT; j++) red[(((wr - 1) * WM + wm) * MTW * NT + i * NT + j) * 64 + l] = acc[i][j];
        }
        __syncthreads();
        if (wr == 0) {
            for (int r = 1; r < WR; r++)
#pragma unroll
                for (int i = 0; i < MTW; i++)
#pragma unroll
                    for (int j = 0; j < NT; j++) acc[i][j] += red[(((r - 1) * WM + wm) * MTW * NT + i * NT + j) * 64 + l];
        }
    }
    if (wr == 0) {
        double* out = part + (int64_t)blockIdx.x * (16 * MT) * (16 * NT);
#pragma unroll
        for (int i = 0; i < MTW; i++)
#pragma unroll
            for (int j = 0; j < NT; j++)
#pragma unroll
                for (int v = 0; v < 4; v++) {
                    const int row = 16 * (wm * MTW + i) + drow(l, v);
                    out[row * (16 * NT) + 16 * j + cl] = acc[i][j][v];
                }
    }
}

// out[i] = sum over parts of part[p][i] in a fixed order (deterministic).
// A workgroup owns 64 consecutive elements (one per lane) and its 16
// wavefronts each sum a contiguous range of the parts, so every load of a
// wavefront is one coalesced 512-byte row piece and the whole chip takes
// part; the 16 range sums are added in LDS in range order.
constexpr int RED_WAVES = 16;

__global__ __launch_bounds__(64 * RED_WAVES) void k_reduce_parts(int nparts, int64_t elems,
                                                                 const double* __restrict__ part,
                                                                 double* __restrict__ out) {
    __shared__ double red[RED_WAVES][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t i = (int64_t)blockIdx.x * 64 + lane;
    const int per = (nparts + RED_WAVES - 1) / RED_WAVES;
    const int p0 = min(nparts, w * per), p1 = min(nparts, p0 + per);
    double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (i < elems) {
        int p = p0;
        for (; p + 8 <= p1; p += 8)
#pragma unroll
            for (int u = 0; u < 8; u++) s[u] += part[(int64_t)(p + u) * elems + i];
        for (; p < p1; p++) s[0] += part[(int64_t)p * elems + i];
    }
    red[w][lane] = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
    __syncthreads();
    if (w == 0 && i < elems) {
        double t = red[0][lane];
#pragma unroll
        for (int q = 1; q < RED_WAVES; q++) t += red[q][lane];
        out[i] = t;
    }
}

// D = alpha op(A) op(B) + beta C for small matrices, one thread per output.
// op(A) is M x K: A[i*lda + p] (or A[p*lda + i] if ta); op(B) is K x N.
// C may alias D (elementwise read-then-write by the same thread).  The
// operand strides are fixed before the loop, so the unrolled body has no
// branches and issues the loads of 16 steps ahead of their FMAs (the sum
// is still taken in order p = 0, 1, ...).
__global__ void k_small_gemm(int M, int N, int K, double alpha, const double* __restrict__ A,
                             int64_t lda, int ta, const double* __restrict__ B, int64_t ldb,
                             int tb, double beta, const double* C, int64_t ldc, double* D,
                             int64_t ldd) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)M * N) return;
    const int i = (int)(t / N), j = (int)(t % N);
    const int64_t ap = ta ? lda : 1, bp = tb ? 1 : ldb;
    const double* a_row = A + (ta ? (int64_t)i : (int64_t)i * lda);
    const double* b_col = B + (tb ? (int64_t)j * ldb : (int64_t)j);
    double s = 0.0;
#pragma unroll 16
    for (int p = 0; p < K; p++) s = fma(a_row[p * ap], b_col[p * bp], s);
    double r = alpha * s;
    if (beta != 0.0) r = fma(beta, C[(int64_t)i * ldc + j], r);
    D[(int64_t)i * ldd + j] = r;
}

// In-place solve with a lower-triangular L (n x n, ld ldl, n <= 128) on
// B (n x m):
//   trans == 0:  L X = B   (forward substitution)
//   trans == 1:  L^T X = B (backward substitution; L^T is upper)
// One 64-lane workgroup per column of B (the columns are independent); lane
// l keeps rows l and l + 64 of its column in registers.  Column-oriented
// substitution: at step i the owner lane finishes x_i (one multiply by the
// reciprocal of L_ii, computed up front), it is broadcast with v_readlane,
// and every lane removes its contribution from its own rows with one FMA.  The coefficients do not depend on x, so the
// unrolled loop issues their loads ahead; no shared memory is used.
constexpr int TRSM_NMAX = 128;

template <int TRANS>
__global__ __launch_bounds__(64) void k_trsm_lower(int n, int m, const double* __restrict__ L,
                                                   int64_t ldl, double* B, int64_t ldb) {
    const int l = threadIdx.x, j = blockIdx.x;
    const int r0 = l, r1 = l + 64;
    // rows clamped into the n x n block for the loads (values masked)
    const int c0r = (r0 < n) ? r0 : n - 1, c1r = (r1 < n) ? r1 : n - 1;
    double x0 = (r0 < n) ? B[(int64_t)r0 * ldb + j] : 0.0;
    double x1 = (r1 < n) ? B[(int64_t)r1 * ldb + j] : 0.0;
    // reciprocals of the diagonal entries of the lane's own rows, off the
    // dependency chain of the substitution
    const double rd0 = 1.0 / L[(int64_t)c0r * ldl + c0r];
    const double rd1 = 1.0 / L[(int64_t)c1r * ldl + c1r];
    // 16 steps at a time: all their coefficient loads first (clamped, so
    // unconditional), then the substitution steps, which have no branch
    constexpr int U = 16;
    for (int it0 = 0; it0 < n; it0 += U) {
        double a0[U], a1[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int itc = (it0 + u < n) ? it0 + u : n - 1;
            const int i = TRANS ? (n - 1 - itc) : itc;
            // coefficient of x_i in rows r0, r1: L[r][i] (forward) or
            // L^T[r][i] = L[i][r] (backward)
            a0[u] = TRANS ? L[(int64_t)i * ldl + c0r] : L[(int64_t)c0r * ldl + i];
            a1[u] = TRANS ? L[(int64_t)i * ldl + c1r] : L[(int64_t)c1r * ldl + i];
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            const bool valid = it0 + u < n;  // uniform
            const int itc = valid ? it0 + u : n - 1;
            const int i = TRANS ? (n - 1 - itc) : itc;
            // rows below (forward) or above (backward) the pivot take part
            const bool t0 = valid && (TRANS ? r0 < i : (r0 > i && r0 < n));
            const bool t1 = valid && (TRANS ? r1 < i : (r1 > i && r1 < n));
            x0 = (valid && l == i) ? x0 * rd0 : x0;
            x1 = (valid && l + 64 == i) ? x1 * rd1 : x1;
            const double xi = bcast((i < 64) ? x0 : x1, i & 63);
            x0 -= (t0 ? a0[u] : 0.0) * xi;
            x1 -= (t1 ? a1[u] : 0.0) * xi;
        }
    }
    if (r0 < n) B[(int64_t)r0 * ldb + j] = x0;
    if (r1 < n) B[(int64_t)r1 * ldb + j] = x1;
}

__global__ __launch_bounds__(1024) void k_qr_top(int n, const double* __restrict__ Vt, int64_t ldv,
                                                 double* __restrict__ P, double* __restrict__ T) {
    extern __shared__ double sm[];
    qr_top_body(n, Vt, ldv, P, T, sm);
}

// Phase-normalize the top-level R (k x k, rows of ld KP in Rin) and write
//   Rout = D Rin (upper part, zero below), G0 = D (KP x KP, zero padded),
// where D = diag(sign(R_jj)) with sign(0) = +1.
__global__ void k_finish_r(int k, int KP, const double* __restrict__ Rin, int64_t ldri,
                           double* __restrict__ Rout, int64_t ldr, double* __restrict__ G0) {
    const int tid = threadIdx.x;
    for (int e = tid; e < k * k; e += blockDim.x) {
        const int i = e / k, j = e % k;
        const double d = (Rin[(int64_t)i * ldri + i] < 0.0) ? -1.0 : 1.0;
        Rout[(int64_t)i * ldr + j] = (j >= i) ? d * Rin[(int64_t)i * ldri + j] : 0.0;
    }
    for (int e = tid; e < KP * KP; e += blockDim.x) {
        const int i = e / KP, j = e % KP;
        double v = 0.0;
        if (i == j && i < k) v = (Rin[(int64_t)i * ldri + i] < 0.0) ? -1.0 : 1.0;
        G0[e] = v;
    }
}

// prod[c] = N_c G_c (K0P x KP): N_c^T is stored (KP x K0P) in NcT[c]; G_c
// is KP x KP, rows of ld ldg starting at row c*grow_stride of Gbase (only
// the first k rows/cols are meaningful).  One block per chunk; both small
// operands are staged in LDS.  Each thread owns 4 x 4 patches of the output
// (rows 4*pi .. 4*pi+3, columns pj + (KP/4)*c), so one LDS read serves four
// FMAs; every output is summed over p in order.  K0P and KP are multiples of
// 16.
__global__ __launch_bounds__(256) void k_chunk_prod(int K0P, int KP, int k, const double* __restrict__ NcT,
                             const double* __restrict__ Gbase, int64_t ldg, int64_t grow_stride,
                             double* __restrict__ prod) {
    __shared__ double Ns[64 * 129];  // N_c^T, KP x (K0P + 1)
    __shared__ double Gs[64 * 65];   // G_c,   KP x (KP + 1)
    const int c = blockIdx.x;
    const double* NT = NcT + (int64_t)c * KP * K0P;
    const double* G = Gbase + (int64_t)c * grow_stride * ldg;
    double* out = prod + (int64_t)c * K0P * KP;
    for (int e = threadIdx.x; e < KP * K0P; e += blockDim.x) Ns[(e / K0P) * (K0P + 1) + e % K0P] = NT[e];
    for (int e = threadIdx.x; e < KP * KP; e += blockDim.x) {
        const int i = e / KP, j = e % KP;
        Gs[i * (KP + 1) + j] = (i < k && j < k) ? G[(int64_t)i * ldg + j] : 0.0;
    }
    __syncthreads();
    const int CQ = KP / 4, npatch = (K0P / 4) * CQ;
    for (int pe = threadIdx.x; pe < npatch; pe += blockDim.x) {
        const int pi = pe / CQ, pj = pe % CQ;
        double acc[4][4];
#pragma unroll
        for (int r = 0; r < 4; r++)
#pragma unroll
            for (int c = 0; c < 4; c++) acc[r][c] = 0.0;
        for (int p = 0; p < k; p++) {
            double a[4], b[4];
#pragma unroll
            for (int r = 0; r < 4; r++) a[r] = Ns[p * (K0P + 1) + 4 * pi + r];
#pragma unroll
            for (int c = 0; c < 4; c++) b[c] = Gs[p * (KP + 1) + pj + CQ * c];
#pragma unroll
            for (int r = 0; r < 4; r++)
#pragma unroll
                for (int c = 0; c < 4; c++) acc[r][c] = fma(a[r], b[c], acc[r][c]);
        }
#pragma unroll
        for (int r = 0; r < 4; r++)
#pragma unroll
            for (int c = 0; c < 4; c++) out[(4 * pi + r) * KP + pj + CQ * c] = acc[r][c];
    }
}

// dst[(s*CT + ct)*64 + l] = src[rows_kidx(s, l/16)*KP + 16*ct + l%16]: a
// K0P x KP matrix in the order in which 64 lanes read it as the B operand
// of FP64 MFMA K-steps whose K index is split as rows_kidx(s, l/16).
__global__ void k_permute_b(int K0P, int KP, const double* __restrict__ src, double* __restrict__ dst) {
    const int n = K0P * KP, CT = KP / 16;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
        const int l = e & 63, sc = e >> 6, s = sc / CT, ct = sc % CT;
        dst[e] = src[rows_kidx(s, l >> 4) * KP + 16 * ct + (l & 15)];
    }
}

// D = a op(X) + b op(Y) + c I (M x N), masked: mode 1 keeps j <= i, mode 2
// keeps j >= i, mode 3 mirrors the lower part to the upper (copyltu).
__global__ void k_small_ew(int M, int N, double a, const double* __restrict__ X, int64_t ldx, int tx, double b,
                           const double* __restrict__ Y, int64_t ldy, int ty, double c, int mode, double* D,
                           int64_t ldd) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)M * N) return;
    const int i = (int)(t / N), j = (int)(t % N);
    int si = i, sj = j;
    if (mode == 3 && j > i) { si = j; sj = i; }
    double v = 0.0;
    if (X) v += a * (tx ? X[(int64_t)sj * ldx + si] : X[(int64_t)si * ldx + sj]);
    if (Y) v += b * (ty ? Y[(int64_t)sj * ldy + si] : Y[(int64_t)si * ldy + sj]);
    if (si == sj) v += c;
    if ((mode == 1 && j > i) || (mode == 2 && j < i)) v = 0.0;
    D[(int64_t)i * ldd + j] = v;
}

// ---------------------------------------------------------------- launchers

hipError_t launch_small_ew(int M, int N, double a, const double* X, int64_t ldx, int tx, double b, const double* Y,
                           int64_t ldy, int ty, double c, int mode, double* D, int64_t ldd, hipStream_t st) {
    if (M <= 0 || N <= 0) return hipSuccess;
    const int64_t nb = ((int64_t)M * N + 255) / 256;
    hipLaunchKernelGGL(k_small_ew, dim3((unsigned)nb), dim3(256), 0, st, M, N, a, X, ldx, tx, b, Y, ldy, ty, c, mode,
                       D, ldd);
    return hipGetLastError();
}

#define XTY_CASE(MT, NT, WM)                                                               \
    if (mt == MT && nt == NT) {                                                             \
        hipLaunchKernelGGL((k_xty_partial<MT, NT, WM>), dim3(nblk), dim3(256), 0, st, nrows, X, \
                           ldx, p, Y, ldy, q, rows_per_blk, part);                          \
        return hipGetLastError();                                                           \
    }

hipError_t launch_xty3_partial(int mt, int nb, int64_t nrows, const double* X, int64_t ldx, int p, const double* Y0,
                               int64_t ld0, const double* Y1, int64_t ld1, const double* Y2, int64_t ld2, int q,
                               int nblk, int64_t rows_per_blk, double* part, hipStream_t st) {
#define XTY3_CASE(MT, NB)                                                                                      \
    if (mt == MT && nb == NB) {                                                                                \
        hipLaunchKernelGGL((k_xty3_partial<MT, NB>), dim3(nblk), dim3(256), 0, st, nrows, X, ldx, p, Y0, ld0, Y1, \
                           ld1, Y2, ld2, q, rows_per_blk, part);                                               \
        return hipGetLastError();                                                                              \
    }
    XTY3_CASE(1, 1)
    XTY3_CASE(1, 2)
    XTY3_CASE(1, 4)
    XTY3_CASE(2, 1)
    XTY3_CASE(2, 2)
    XTY3_CASE(2, 4)
    XTY3_CASE(4, 1)
    XTY3_CASE(4, 2)
    XTY3_CASE(4, 4)
    XTY3_CASE(8, 1)
    XTY3_CASE(8, 2)
    XTY3_CASE(8, 4)
#undef XTY3_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_xty_partial(int mt, int nt, int64_t nrows, const double* X, int64_t ldx, int p,
                              const double* Y, int64_t ldy, int q, int nblk, int64_t rows_per_blk,
                              double* part, hipStream_t st) {
    XTY_CASE(1, 1, 1)
    XTY_CASE(1, 2, 1)
    XTY_CASE(1, 4, 1)
    XTY_CASE(2, 1, 2)
    XTY_CASE(2, 2, 2)
    XTY_CASE(2, 4, 2)
    XTY_CASE(4, 1, 4)
    XTY_CASE(4, 2, 4)
    XTY_CASE(4, 4, 4)
    XTY_CASE(8, 1, 4)
    XTY_CASE(8, 2, 4)
    XTY_CASE(8, 4, 4)
    return hipErrorInvalidValue;
}

hipError_t launch_reduce_parts(int nparts, int64_t elems, const double* part, double* out,
                               hipStream_t st) {
    if (elems <= 0) return hipSuccess;
    const int64_t nb = (elems + 63) / 64;
    hipLaunchKernelGGL(k_reduce_parts, dim3((unsigned)nb), dim3(64 * RED_WAVES), 0, st, nparts, elems, part,
                       out);
    return hipGetLastError();
}

hipError_t launch_small_gemm(int M, int N, int K, double alpha, const double* A, int64_t lda, int ta,
                             const double* B, int64_t ldb, int tb, double beta, const double* C,
                             int64_t ldc, double* D, int64_t ldd, hipStream_t st) {
    if (M <= 0 || N <= 0) return hipSuccess;
    const int bs = 256;
    const int64_t nb = ((int64_t)M * N + bs - 1) / bs;
    hipLaunchKernelGGL(k_small_gemm, dim3((unsigned)nb), dim3(bs), 0, st, M, N, K, alpha, A, lda, ta,
                       B, ldb, tb, beta, C, ldc, D, ldd);
    return hipGetLastError();
}

hipError_t launch_trsm_lower(int n, int m, const double* L, int64_t ldl, int trans, double* B,
                             int64_t ldb, hipStream_t st) {
    if (n <= 0 || m <= 0) return hipSuccess;
    if (n > TRSM_NMAX) return hipErrorInvalidValue;
    if (trans) hipLaunchKernelGGL(k_trsm_lower<1>, dim3(m), dim3(64), 0, st, n, m, L, ldl, B, ldb);
    else hipLaunchKernelGGL(k_trsm_lower<0>, dim3(m), dim3(64), 0, st, n, m, L, ldl, B, ldb);
    return hipGetLastError();
}

hipError_t launch_qr_top(int n, const double* Vt, int64_t ldv, double* P, double* T, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const size_t shm = (size_t)qr_top_lds(n) * sizeof(double);
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void*)k_qr_top, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           160 * 1024);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL(k_qr_top, dim3(1), dim3(1024), shm, st, n, Vt, ldv, P, T);
    return hipGetLastError();
}

hipError_t launch_finish_r(int k, int KP, const double* Rin, int64_t ldri, double* Rout, int64_t ldr,
                           double* G0, hipStream_t st) {
    hipLaunchKernelGGL(k_finish_r, dim3(1), dim3(256), 0, st, k, KP, Rin, ldri, Rout, ldr, G0);
    return hipGetLastError();
}

hipError_t launch_permute_b(int K0P, int KP, const double* src, double* dst, hipStream_t st) {
    hipLaunchKernelGGL(k_permute_b, dim3((K0P * KP + 255) / 256), dim3(256), 0, st, K0P, KP, src, dst);
    return hipGetLastError();
}


hipError_t launch_chunk_prod(int nchunk, int K0P, int KP, int k, const double* Nc, const double* Gbase,
                             int64_t ldg, int64_t grow_stride, double* prod, hipStream_t st) {
    hipLaunchKernelGGL(k_chunk_prod, dim3(nchunk), dim3(256), 0, st, K0P, KP, k, Nc, Gbase, ldg,
                       grow_stride, prod);
    return hipGetLastError();
}

}  // namespace tho
