// Complex (complex128, interleaved re/im) kernels of libtho for gfx950.
//
// The panel products of the complex path (V^H A, A + V Z, V^H Q_, Q_ + V N)
// run on the real FP64 MFMA kernels through real views of the interleaved
// data (see tho_complex.cpp); this file holds what is genuinely complex:
//   - the chunked tall-skinny Householder QR (leaf) and the formation of Q
//     (form), LDS-resident tiles, one workgroup per chunk;
//   - the QR of the k0 x k0 top block of V (second choice of P), triangular
//     solves with T, small products with conjugate transposes;
//   - re/im combination of the real-view reductions and the expansion of a
//     small complex matrix into its real 2 x 2 block form.
// Reflectors follow the complex LAPACK convention: H = I - tau u u^H with
// u_j = 1, beta = -sign(Re alpha) ||x|| real, tau = (beta - alpha) / beta,
// u = x / (alpha - beta); a zero subcolumn with real alpha gives tau = 0.
// H^H is applied to the matrix being factored; the formation applies H.
#include "tho_device.h"
#include "tho_internal.h"

namespace tho {

namespace {

using cplx = dcplx;
__device__ __forceinline__ cplx cmk(double r, double i) { return {r, i}; }
__device__ __forceinline__ cplx cadd(cplx a, cplx b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cplx csub(cplx a, cplx b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cplx cmul(cplx a, cplx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
// conj(a) * b
__device__ __forceinline__ cplx cmulc(cplx a, cplx b) { return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re}; }
__device__ __forceinline__ cplx cconj(cplx a) { return {a.re, -a.im}; }
__device__ __forceinline__ cplx cscale(cplx a, double s) { return {a.re * s, a.im * s}; }
__device__ __forceinline__ cplx cdiv(cplx a, cplx b) {
    const double d = b.re * b.re + b.im * b.im;
    return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}
__device__ __forceinline__ double cabs2(cplx a) { return a.re * a.re + a.im * a.im; }

constexpr int CW = 256;  // threads per workgroup of the complex kernels

// Workgroup sum (all threads receive it); `red` holds CW / 64 doubles.
__device__ double wg_sum(double x, double* red) {
    x = sum_wave(x);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = x;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < CW / 64; i++) s += red[i];
    return s;
}

// Reflector from alpha and sigma^2 = ||x_sub||^2.
__device__ __forceinline__ void make_reflector(cplx alpha, double sig2, double& beta, cplx& tau, cplx& scale) {
    if (sig2 == 0.0 && alpha.im == 0.0) {
        beta = alpha.re;
        tau = cmk(0.0, 0.0);
        scale = cmk(0.0, 0.0);
        return;
    }
    const double nrm = sqrt(cabs2(alpha) + sig2);
    beta = (alpha.re < 0.0) ? nrm : -nrm;
    tau = cmk((beta - alpha.re) / beta, -alpha.im / beta);
    scale = cdiv(cmk(1.0, 0.0), cmk(alpha.re - beta, alpha.im));
}

// ---------------------------------------------------------------------------
// Leaf: per chunk, tiles of TBC rows; tile 0 plain QR, tile t > 0 QR of
// [R; X_t] with u_j = [e_j; y_j].  Tiles, R and the Gram of the vectors live
// in LDS (complex, row stride KP + 1).  Output: vectors into Y (tile rows;
// tile 0 stores U_0 explicitly, unit diagonal and zeros above), T_t (upper,
// H_0...H_{k-1} = I - U T U^H) and tau into per-tile storage, and the chunk's
// R into rows c*k .. of Rnext.
// ---------------------------------------------------------------------------
template <int KP, int TBC>
__global__ __launch_bounds__(CW) void k_zleaf(ZLevel L) {
    extern __shared__ double smd[];
    constexpr int LD = KP + 1;
    cplx* Xs = (cplx*)smd;          // TBC x LD
    cplx* Rs = Xs + TBC * LD;       // KP x LD: running R
    cplx* Gs = Rs + KP * LD;        // KP x LD: Gram, then T
    cplx* taus = Gs + KP * LD;      // KP
    cplx* wv = taus + KP;           // KP: w_c of the current column
    double* red = (double*)(wv + KP);  // 8 doubles + misc
    cplx* sc = (cplx*)(red + 8);    // 2: tau, scale of the current column
    const int tid = threadIdx.x;
    const int c = blockIdx.x;
    const int k = L.k;
    const int64_t cr0 = (int64_t)c * L.m / L.nchunk;
    const int64_t cr1 = (int64_t)(c + 1) * L.m / L.nchunk;
    const int ntiles = (int)((cr1 - cr0 + TBC - 1) / TBC);
    for (int e = tid; e < KP * LD; e += CW) Rs[e] = cmk(0.0, 0.0);
    for (int t = 0; t < ntiles; t++) {
        const int64_t r0 = cr0 + (int64_t)t * TBC;
        const int trows = (int)((cr1 - r0 < TBC) ? (cr1 - r0) : TBC);
        const bool plain = (t == 0);
        const cplx* X = L.X + r0 * L.ldx;
        cplx* Y = L.Y + r0 * L.ldy;
        __syncthreads();
        for (int e = tid; e < TBC * KP; e += CW) {
            const int i = e / KP, j = e % KP;
            Xs[i * LD + j] = (i < trows && j < k) ? X[(int64_t)i * L.ldx + j] : cmk(0.0, 0.0);
        }
        __syncthreads();
        for (int j = 0; j < k; j++) {
            // sigma^2 over the sub rows (plain: rows > j of the tile; structured: all tile rows)
            double ss = 0.0;
            for (int i = tid; i < trows; i += CW)
                if (!plain || i > j) ss += cabs2(Xs[i * LD + j]);
            ss = wg_sum(ss, red);
            if (tid == 0) {
                cplx alpha = plain ? Xs[j * LD + j] : Rs[j * LD + j];
                double beta;
                cplx tau, scl;
                make_reflector(alpha, ss, beta, tau, scl);
                sc[0] = tau;
                sc[1] = scl;
                taus[j] = tau;
                if (plain) Xs[j * LD + j] = cmk(beta, 0.0);
                else Rs[j * LD + j] = cmk(beta, 0.0);
            }
            __syncthreads();
            const cplx tau = sc[0], scl = sc[1];
            for (int i = tid; i < trows; i += CW)
                if (!plain || i > j) Xs[i * LD + j] = cmul(Xs[i * LD + j], scl);
            __syncthreads();
            // w_c = (pivot row)_c + sum_sub conj(u_i) X[i][c], c > j
            const int ncol = k - j - 1;
            if (ncol > 0) {
                const int groups = CW / KP;  // row groups per column
                const int cc = j + 1 + (tid % KP), g = tid / KP;
                cplx s = cmk(0.0, 0.0);
                if (cc < k)
                    for (int i = g; i < trows; i += groups)
                        if (!plain || i > j) s = cadd(s, cmulc(Xs[i * LD + j], Xs[i * LD + cc]));
                // reduce over groups through Gs scratch rows (Gs is rebuilt after the loop)
                Gs[g * LD + (tid % KP)] = s;
                __syncthreads();
                if (tid < KP && j + 1 + tid < k) {
                    cplx a = plain ? Xs[j * LD + j + 1 + tid] : Rs[j * LD + j + 1 + tid];
                    for (int q = 0; q < groups; q++) a = cadd(a, Gs[q * LD + tid]);
                    wv[j + 1 + tid] = a;
                }
                __syncthreads();
                // pivot row and sub rows -= conj(tau) u w_c
                const cplx tc = cconj(tau);
                for (int e = tid; e < (trows + 1) * ncol; e += CW) {
                    const int i = e / ncol - 1, cc2 = j + 1 + e % ncol;  // i = -1: pivot row
                    const cplx tw = cmul(tc, wv[cc2]);
                    if (i < 0) {
                        if (plain) Xs[j * LD + cc2] = csub(Xs[j * LD + cc2], tw);
                        else Rs[j * LD + cc2] = csub(Rs[j * LD + cc2], tw);
                    } else if (!plain || i > j) {
                        Xs[i * LD + cc2] = csub(Xs[i * LD + cc2], cmul(Xs[i * LD + j], tw));
                    }
                }
                __syncthreads();
            }
        }
        __syncthreads();
        // plain tile: R from the tile's upper part; U_0 with explicit unit diagonal
        if (plain) {
            for (int e = tid; e < KP * KP; e += CW) {
                const int i = e / KP, j = e % KP;
                if (i < k && j < k) Rs[i * LD + j] = (j >= i) ? Xs[i * LD + j] : cmk(0.0, 0.0);
            }
            __syncthreads();
            for (int e = tid; e < TBC * KP; e += CW) {
                const int i = e / KP, j = e % KP;
                if (i < k && j < KP) Xs[i * LD + j] = (j < i) ? Xs[i * LD + j] : cmk(j == i ? 1.0 : 0.0, 0.0);
            }
            __syncthreads();
        }
        // Gram of the vectors: plain u_p^H u_i over the tile; structured y_p^H y_i
        for (int e = tid; e < KP * KP; e += CW) {
            const int p = e / KP, i = e % KP;
            cplx s = cmk(0.0, 0.0);
            if (p < i && i < k)
                for (int r = 0; r < trows; r++) s = cadd(s, cmulc(Xs[r * LD + p], Xs[r * LD + i]));
            Gs[p * LD + i] = s;
        }
        __syncthreads();
        // T: T(i,i) = tau_i, T(0:i, i) = -tau_i T(0:i, 0:i) G(0:i, i); rows are independent
        if (tid < k) {
            // fully unrolled so that Trow stays in registers
            const int r = tid;
            cplx Trow[KP];
#pragma unroll
            for (int j = 0; j < KP; j++) Trow[j] = (j == r) ? taus[r] : cmk(0.0, 0.0);
#pragma unroll
            for (int i = 1; i < KP; i++) {
                if (i > r && i < k) {
                    cplx s = cmk(0.0, 0.0);
#pragma unroll
                    for (int p = 0; p < i; p++)
                        if (p >= r) s = cadd(s, cmul(Trow[p], Gs[p * LD + i]));
                    Trow[i] = cmul(cmk(-taus[i].re, -taus[i].im), s);
                }
            }
            cplx* Tt = L.Tt + ((int64_t)c * L.maxtiles + t) * KP * KP;
#pragma unroll
            for (int j = 0; j < KP; j++) Tt[r * KP + j] = (j < k) ? Trow[j] : cmk(0.0, 0.0);
        }
        // vectors into Y
        for (int e = tid; e < TBC * KP; e += CW) {
            const int i = e / KP, j = e % KP;
            if (i < trows && j < k) Y[(int64_t)i * L.ldy + j] = Xs[i * LD + j];
        }
    }
    __syncthreads();
    for (int e = tid; e < k * KP; e += CW) {
        const int i = e / KP, j = e % KP;
        L.Rnext[((int64_t)c * k + i) * L.ldrn + j] = (j < k && j >= i) ? Rs[i * LD + j] : cmk(0.0, 0.0);
    }
}

// Formation: chunk c's rows of Q = Q_chunk G_c, tiles last to first, C in LDS:
//   structured tile t:  K = T_t C,                rows = -Y_t K,  C <- C - K
//   plain tile 0:       K = T_0 (U_0[0:k]^H C),   rows = [C; 0] - U_0 K
// A thread owns a whole output row (reads its vector row, then overwrites it).
template <int KP, int TBC>
__global__ __launch_bounds__(CW) void k_zform(ZLevel L) {
    extern __shared__ double smd[];
    constexpr int LD = KP + 1;
    cplx* Cs = (cplx*)smd;      // KP x LD
    cplx* Ks = Cs + KP * LD;    // KP x LD
    cplx* Es = Ks + KP * LD;    // KP x LD
    cplx* Ts = Es + KP * LD;    // KP x LD
    const int tid = threadIdx.x;
    const int c = blockIdx.x;
    const int k = L.k;
    const int64_t cr0 = (int64_t)c * L.m / L.nchunk;
    const int64_t cr1 = (int64_t)(c + 1) * L.m / L.nchunk;
    const int ntiles = (int)((cr1 - cr0 + TBC - 1) / TBC);
    {
        const cplx* G = L.Gin + (int64_t)c * L.gstride * L.ldg;
        for (int e = tid; e < KP * KP; e += CW) {
            const int i = e / KP, j = e % KP;
            Cs[i * LD + j] = (i < k && j < k) ? G[(int64_t)i * L.ldg + j] : cmk(0.0, 0.0);
        }
    }
    for (int t = ntiles - 1; t >= 0; t--) {
        const int64_t r0 = cr0 + (int64_t)t * TBC;
        const int trows = (int)((cr1 - r0 < TBC) ? (cr1 - r0) : TBC);
        const bool plain = (t == 0);
        cplx* Y = L.Y + r0 * L.ldy;
        const cplx* Tt = L.Tt + ((int64_t)c * L.maxtiles + t) * KP * KP;
        __syncthreads();
        for (int e = tid; e < KP * KP; e += CW) Ts[(e / KP) * LD + e % KP] = Tt[e];
        // plain: E = U_0[0:k]^H C, else E = C
        for (int e = tid; e < KP * KP; e += CW) {
            const int i = e / KP, j = e % KP;
            cplx s = cmk(0.0, 0.0);
            if (i < k && j < k) {
                if (plain) {
                    for (int p = 0; p < k; p++) s = cadd(s, cmulc(Y[(int64_t)p * L.ldy + i], Cs[p * LD + j]));
                } else {
                    s = Cs[i * LD + j];
                }
            }
            Es[i * LD + j] = s;
        }
        __syncthreads();
        // K = T E
        for (int e = tid; e < KP * KP; e += CW) {
            const int i = e / KP, j = e % KP;
            cplx s = cmk(0.0, 0.0);
            if (i < k && j < k)
                for (int p = i; p < k; p++) s = cadd(s, cmul(Ts[i * LD + p], Es[p * LD + j]));
            Ks[i * LD + j] = s;
        }
        __syncthreads();
        for (int i = tid; i < trows; i += CW) {
            cplx* yr = Y + (int64_t)i * L.ldy;
            cplx yv[KP];
#pragma unroll
            for (int p = 0; p < KP; p++) yv[p] = (p < k) ? yr[p] : cmk(0.0, 0.0);
            for (int j = 0; j < k; j++) {
                cplx s = (plain && i < k) ? Cs[i * LD + j] : cmk(0.0, 0.0);
#pragma unroll
                for (int p = 0; p < KP; p++) s = csub(s, cmul(yv[p], Ks[p * LD + j]));
                yr[j] = s;
            }
        }
        __syncthreads();
        if (!plain)
            for (int e = tid; e < KP * KP; e += CW) {
                const int i = e / KP, j = e % KP;
                Cs[i * LD + j] = csub(Cs[i * LD + j], Ks[i * LD + j]);
            }
    }
}

// ---------------------------------------------------------------------------
// QR of the square top block (n <= 64) with real nonnegative diag(R1):
// P = -Q1, T = I + R1^H (lower).  One workgroup, LDS.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(CW) void k_zqr_top(int n, const cplx* __restrict__ Vt, int64_t ldv, cplx* P, cplx* T) {
    extern __shared__ double smd[];
    const int ld = n + 1;
    cplx* M = (cplx*)smd;        // n x ld
    cplx* taus = M + n * ld;     // n
    cplx* wv = taus + n;         // n
    cplx* sc = wv + n;           // 2
    cplx* ub = sc + 2;           // n: the reflector being applied in the formation
    double* red = (double*)(ub + n);  // 8
    double* sgn = red + 8;       // n
    const int tid = threadIdx.x;
    for (int e = tid; e < n * n; e += CW) M[(e / n) * ld + e % n] = Vt[(int64_t)(e / n) * ldv + e % n];
    __syncthreads();
    // Two workgroup barriers per column: a quad of lanes per column c >= j
    // forms d_c = sum_{i > j} conj(x_ij) x_ic (c = j gives sigma^2); after the
    // barrier every thread builds the reflector itself and the quads of the
    // columns c > j apply it, w_c = M[j][c] + conj(s) d_c with u = [1; s x_sub];
    // the pivot-row entries and the scaled column j are stored after the
    // second barrier (no later step of the factorization reads them before).
    for (int j = 0; j < n; j++) {
        const int cc = j + (tid >> 2), q = tid & 3;
        double dr = 0.0, di = 0.0;
        if (cc < n)
            for (int i = j + 1 + q; i < n; i += 4) {
                const cplx a = M[i * ld + j], b = M[i * ld + cc];
                dr += a.re * b.re + a.im * b.im;
                di += a.re * b.im - a.im * b.re;
            }
        dr = sum_quad(dr);
        di = sum_quad(di);
        if (cc < n && q == 0) wv[cc] = cmk(dr, di);
        __syncthreads();
        const cplx alpha = M[j * ld + j];
        double beta;
        cplx tau, scl;
        make_reflector(alpha, wv[j].re, beta, tau, scl);
        cplx rowj = cmk(0.0, 0.0);
        if (cc > j && cc < n) {
            const cplx d = wv[cc];
            rowj = M[j * ld + cc];
            // w = p + conj(s) d ; the column takes -conj(tau) w u
            const cplx w = cadd(rowj, cmulc(scl, d));
            const cplx tw = cmul(cconj(tau), w);
            const cplx tws = cmul(tw, scl);
            rowj = csub(rowj, tw);
            for (int i = j + 1 + q; i < n; i += 4) M[i * ld + cc] = csub(M[i * ld + cc], cmul(M[i * ld + j], tws));
        }
        __syncthreads();
        if (cc > j && cc < n && q == 0) M[j * ld + cc] = rowj;
        for (int i = j + 1 + tid; i < n; i += CW) M[i * ld + j] = cmul(M[i * ld + j], scl);
        if (tid == 0) {
            taus[j] = tau;
            M[j * ld + j] = cmk(beta, 0.0);
        }
    }
    __syncthreads();
    // T = I + D R^H (lower), D = sign(diag R) real; keep the signs
    for (int e = tid; e < n * n; e += CW) {
        const int i = e / n, jj = e % n;
        cplx v = cmk(i == jj ? 1.0 : 0.0, 0.0);
        if (jj <= i) {
            const double d = (M[jj * ld + jj].re < 0.0) ? -1.0 : 1.0;
            const cplx r = M[jj * ld + i];  // R[jj][i]
            v = cadd(v, cmk(d * r.re, -d * r.im));
        }
        T[(int64_t)i * n + jj] = v;
    }
    for (int i = tid; i < n; i += CW) sgn[i] = (M[i * ld + i].re < 0.0) ? -1.0 : 1.0;
    __syncthreads();
    // Q in place (backward accumulation): H_j applied to the formed columns
    // c > j, two barriers per column.  The dots copy u_j into ub, so that the
    // update reads it there while column j is overwritten by H_j e_j in the
    // same phase (row j of a formed column c > j is zero).
    for (int j = n - 1; j >= 0; j--) {
        const cplx tau = taus[j];
        if (j < n - 1) {
            {
                // a quad per column
                const int cc = j + 1 + (tid >> 2), q = tid & 3;
                double sr = 0.0, si = 0.0;
                if (cc < n)
                    for (int i = j + 1 + q; i < n; i += 4) {
                        const cplx a = M[i * ld + j], b = M[i * ld + cc];
                        sr += a.re * b.re + a.im * b.im;
                        si += a.re * b.im - a.im * b.re;
                    }
                sr = sum_quad(sr);
                si = sum_quad(si);
                if (cc < n && q == 0) wv[cc] = cmk(sr, si);
            }
            for (int i = j + 1 + tid; i < n; i += CW) ub[i] = M[i * ld + j];
            __syncthreads();
            for (int e = tid; e < (n - j) * (n - j - 1); e += CW) {
                const int i = j + e / (n - j - 1), cc = j + 1 + e % (n - j - 1);
                const cplx u = (i == j) ? cmk(1.0, 0.0) : ub[i];
                M[i * ld + cc] = csub(M[i * ld + cc], cmul(u, cmul(tau, wv[cc])));
            }
        }
        for (int i = tid; i < n; i += CW) {
            if (i > j) M[i * ld + j] = cmul(cmk(-tau.re, -tau.im), ub[i]);
            else if (i == j) M[j * ld + j] = cmk(1.0 - tau.re, -tau.im);
            else M[i * ld + j] = cmk(0.0, 0.0);
        }
        __syncthreads();
    }
    for (int e = tid; e < n * n; e += CW) {
        const int i = e / n, jj = e % n;
        P[(int64_t)i * n + jj] = cscale(M[i * ld + jj], -sgn[jj]);
    }
}

// D = alpha op(A) op(B) + beta C (complex, small); op: 0 none, 1 transpose,
// 2 conjugate transpose.  C may alias D.  The operand strides and the sign
// of the conjugation are fixed before the loop, so the unrolled body has no
// branches and issues the loads of 8 steps ahead (the sum is still taken in
// order p = 0, 1, ...).
__global__ void k_zgemm(int M, int N, int K, cplx alpha, const cplx* A, int64_t lda, int opa, const cplx* B,
                        int64_t ldb, int opb, cplx beta, const cplx* C, int64_t ldc, cplx* D, int64_t ldd) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)M * N) return;
    const int i = (int)(t / N), j = (int)(t % N);
    const int64_t ap = opa ? lda : 1, bp = opb ? 1 : ldb;
    const cplx* a_row = A + (opa ? (int64_t)i : (int64_t)i * lda);
    const cplx* b_col = B + (opb ? (int64_t)j * ldb : (int64_t)j);
    const double sa = (opa == 2) ? -1.0 : 1.0, sb = (opb == 2) ? -1.0 : 1.0;
    cplx s = cmk(0.0, 0.0);
#pragma unroll 8
    for (int p = 0; p < K; p++) {
        const cplx a0 = a_row[p * ap], b0 = b_col[p * bp];
        s = cadd(s, cmul(cmk(a0.re, sa * a0.im), cmk(b0.re, sb * b0.im)));
    }
    cplx r = cmul(alpha, s);
    if (beta.re != 0.0 || beta.im != 0.0) r = cadd(r, cmul(beta, C[(int64_t)i * ldc + j]));
    D[(int64_t)i * ldd + j] = r;
}

// In-place solve with lower-triangular L (n x n, n <= 64) on B (n x m):
//   mode 0: L X = B;  mode 2: L^H X = B.
// One 64-lane workgroup per column of B; lane l keeps row l in registers.
// Column-oriented substitution: at step i the owner lane finishes x_i,
// v_readlane broadcasts it, and every lane whose row depends on x_i removes
// its contribution.  The coefficients do not depend on x, so the unrolled
// loop issues their loads ahead of the substitution; no shared memory.
constexpr int ZTRSM_NMAX = 64;

__global__ __launch_bounds__(64) void k_ztrsm(int n, int m, const cplx* __restrict__ L, int64_t ldl, int mode,
                                              cplx* B, int64_t ldb) {
    const int l = threadIdx.x, j = blockIdx.x;
    const int lc = (l < n) ? l : n - 1;  // row clamped into the block for the loads
    cplx x = (l < n) ? B[(int64_t)l * ldb + j] : cmk(0.0, 0.0);
    const cplx d = L[(int64_t)lc * ldl + lc];
    const cplx dd = mode ? cconj(d) : d;
#pragma unroll 16
    for (int it = 0; it < n; it++) {
        const int i = mode ? (n - 1 - it) : it;
        // coefficient of x_i in row l: L[l][i] (mode 0) or (L^H)[l][i] = conj(L[i][l])
        const cplx a = mode ? cconj(L[(int64_t)i * ldl + lc]) : L[(int64_t)lc * ldl + i];
        if (l == i) x = cdiv(x, dd);
        const cplx xi = cmk(bcast(x.re, i), bcast(x.im, i));
        const bool t = mode ? (l < i) : (l > i && l < n);
        if (t) x = csub(x, cmul(a, xi));
    }
    if (l < n) B[(int64_t)l * ldb + j] = x;
}

// From the real-view reduction Cr = X_ri^T Y_ri (2p x 2q real, ld ldc):
//   out[i][j] = sign * sum_r conj(X[r][i]) Y[r][j]   (p x q complex, ld ldo)
__global__ void k_zcombine(int p, int q, const double* Cr, int64_t ldc, double sign, cplx* out, int64_t ldo) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= p * q) return;
    const int i = t / q, j = t % q;
    const double rr = Cr[(2 * i) * ldc + 2 * j], ri = Cr[(2 * i) * ldc + 2 * j + 1];
    const double ir = Cr[(2 * i + 1) * ldc + 2 * j], ii = Cr[(2 * i + 1) * ldc + 2 * j + 1];
    out[(int64_t)i * ldo + j] = cmk(sign * (rr + ii), sign * (ri - ir));
}

// D = a op(X) + b op(Y) + c I (complex M x N; real a, b, c; op 0 none,
// 1 transpose, 2 conjugate transpose; X or Y may be NULL), masked: mode 1
// keeps j <= i, mode 2 keeps j >= i, mode 3 is copyltu for complex data
// (D_ij for i > j, conj(D_ji) above the diagonal, Re(D_ii) on it).
__global__ void k_zsmall_ew(int M, int N, double a, const cplx* X, int64_t ldx, int opx, double b, const cplx* Y,
                            int64_t ldy, int opy, double c, int mode, cplx* D, int64_t ldd) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)M * N) return;
    const int i = (int)(t / N), j = (int)(t % N);
    const bool mirror = (mode == 3 && j > i);
    const int si = mirror ? j : i, sj = mirror ? i : j;
    auto at = [&](const cplx* P, int64_t ld, int op) {
        const cplx v = op ? P[(int64_t)sj * ld + si] : P[(int64_t)si * ld + sj];
        return (op == 2) ? cconj(v) : v;
    };
    cplx v = cmk(0.0, 0.0);
    if (X) v = cadd(v, cscale(at(X, ldx, opx), a));
    if (Y) v = cadd(v, cscale(at(Y, ldy, opy), b));
    if (si == sj) v.re += c;
    if (mirror) v = cconj(v);
    if (mode == 3 && i == j) v.im = 0.0;
    if ((mode == 1 && j > i) || (mode == 2 && j < i)) v = cmk(0.0, 0.0);
    D[(int64_t)i * ldd + j] = v;
}

// Real 2 x 2 block form of a p x q complex B (ld ldb), scaled by sign:
// dst (2p x 2q, ld 2q) with rows (2i, 2i+1), columns (2j, 2j+1) =
// [[br, bi], [-bi, br]], so that [yr, yi] dst-block = [re, im] of y b.
__global__ void k_zexpand(int p, int q, const cplx* B, int64_t ldb, double sign, double* dst) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= p * q) return;
    const int i = t / q, j = t % q;
    const cplx b = B[(int64_t)i * ldb + j];
    const int ld = 2 * q;
    dst[(2 * i) * ld + 2 * j] = sign * b.re;
    dst[(2 * i) * ld + 2 * j + 1] = sign * b.im;
    dst[(2 * i + 1) * ld + 2 * j] = -sign * b.im;
    dst[(2 * i + 1) * ld + 2 * j + 1] = sign * b.re;
}

// Phase-normalize the top-level R (complex with real diagonal): Rout = D Rin
// (upper), G0 = D (KP x KP), D = diag(sign(Re R_jj)).
__global__ void k_zfinish_r(int k, int KP, const cplx* Rin, int64_t ldri, cplx* Rout, int64_t ldr, cplx* G0) {
    const int tid = threadIdx.x;
    for (int e = tid; e < k * k; e += blockDim.x) {
        const int i = e / k, j = e % k;
        const double d = (Rin[(int64_t)i * ldri + i].re < 0.0) ? -1.0 : 1.0;
        Rout[(int64_t)i * ldr + j] = (j >= i) ? cscale(Rin[(int64_t)i * ldri + j], d) : cmk(0.0, 0.0);
    }
    for (int e = tid; e < KP * KP; e += blockDim.x) {
        const int i = e / KP, j = e % KP;
        double v = 0.0;
        if (i == j && i < k) v = (Rin[(int64_t)i * ldri + i].re < 0.0) ? -1.0 : 1.0;
        G0[e] = cmk(v, 0.0);
    }
}

// Strided complex copy (M x N).
__global__ void k_zcopy(int64_t M, int N, const cplx* src, int64_t lds, cplx* dst, int64_t ldd) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= M * N) return;
    const int64_t i = t / N;
    const int j = (int)(t % N);
    dst[i * ldd + j] = src[i * lds + j];
}

template <int KP>
constexpr int zleaf_tile() { return KP <= 16 ? 256 : (KP <= 32 ? 128 : 64); }

template <int KP>
hipError_t zleaf_t(const ZLevel& L, hipStream_t st) {
    constexpr int TBC = zleaf_tile<KP>();
    constexpr size_t shm = ((size_t)(TBC + 2 * KP) * (KP + 1) + 2 * KP) * sizeof(cplx) + 16 * sizeof(double);
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void*)k_zleaf<KP, TBC>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)shm);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL((k_zleaf<KP, TBC>), dim3(L.nchunk), dim3(CW), shm, st, L);
    return hipGetLastError();
}

template <int KP>
hipError_t zform_t(const ZLevel& L, hipStream_t st) {
    constexpr int TBC = zleaf_tile<KP>();
    constexpr size_t shm = (size_t)4 * KP * (KP + 1) * sizeof(cplx);
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void*)k_zform<KP, TBC>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)shm);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL((k_zform<KP, TBC>), dim3(L.nchunk), dim3(CW), shm, st, L);
    return hipGetLastError();
}

}  // namespace

int ztsqr_tile_rows(int kp) { return kp <= 16 ? 256 : (kp <= 32 ? 128 : 64); }

hipError_t launch_zleaf(int kp, const ZLevel& L, hipStream_t st) {
    if (kp == 16) return zleaf_t<16>(L, st);
    if (kp == 32) return zleaf_t<32>(L, st);
    return hipErrorInvalidValue;
}

hipError_t launch_zform(int kp, const ZLevel& L, hipStream_t st) {
    if (kp == 16) return zform_t<16>(L, st);
    if (kp == 32) return zform_t<32>(L, st);
    return hipErrorInvalidValue;
}

hipError_t launch_zqr_top(int n, const void* Vt, int64_t ldv, void* P, void* T, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    if (n > 64) return hipErrorInvalidValue;
    const size_t shm = ((size_t)n * (n + 1) + 3 * n + 2) * sizeof(cplx) + (8 + n) * sizeof(double);
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void*)k_zqr_top, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           160 * 1024);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL(k_zqr_top, dim3(1), dim3(CW), shm, st, n, (const cplx*)Vt, ldv, (cplx*)P, (cplx*)T);
    return hipGetLastError();
}

hipError_t launch_zgemm(int M, int N, int K, double ar, double ai, const void* A, int64_t lda, int opa, const void* B,
                        int64_t ldb, int opb, double br, double bi, const void* C, int64_t ldc, void* D, int64_t ldd,
                        hipStream_t st) {
    if (M <= 0 || N <= 0) return hipSuccess;
    const int64_t nb = ((int64_t)M * N + 255) / 256;
    hipLaunchKernelGGL(k_zgemm, dim3((unsigned)nb), dim3(256), 0, st, M, N, K, cplx{ar, ai}, (const cplx*)A, lda, opa,
                       (const cplx*)B, ldb, opb, cplx{br, bi}, (const cplx*)C, ldc, (cplx*)D, ldd);
    return hipGetLastError();
}

hipError_t launch_ztrsm(int n, int m, const void* L, int64_t ldl, int mode, void* B, int64_t ldb, hipStream_t st) {
    if (n <= 0 || m <= 0) return hipSuccess;
    if (n > ZTRSM_NMAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_ztrsm, dim3(m), dim3(64), 0, st, n, m, (const cplx*)L, ldl, mode, (cplx*)B, ldb);
    return hipGetLastError();
}

hipError_t launch_zcombine(int p, int q, const double* Cr, int64_t ldc, double sign, void* out, int64_t ldo,
                           hipStream_t st) {
    if (p <= 0 || q <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zcombine, dim3((p * q + 255) / 256), dim3(256), 0, st, p, q, Cr, ldc, sign, (cplx*)out, ldo);
    return hipGetLastError();
}

hipError_t launch_zexpand(int p, int q, const void* B, int64_t ldb, double sign, double* dst, hipStream_t st) {
    if (p <= 0 || q <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zexpand, dim3((p * q + 255) / 256), dim3(256), 0, st, p, q, (const cplx*)B, ldb, sign, dst);
    return hipGetLastError();
}

hipError_t launch_zfinish_r(int k, int KP, const void* Rin, int64_t ldri, void* Rout, int64_t ldr, void* G0,
                            hipStream_t st) {
    hipLaunchKernelGGL(k_zfinish_r, dim3(1), dim3(256), 0, st, k, KP, (const cplx*)Rin, ldri, (cplx*)Rout, ldr,
                       (cplx*)G0);
    return hipGetLastError();
}

hipError_t launch_zsmall_ew(int M, int N, double a, const void* X, int64_t ldx, int opx, double b, const void* Y,
                            int64_t ldy, int opy, double c, int mode, void* D, int64_t ldd, hipStream_t st) {
    if (M <= 0 || N <= 0) return hipSuccess;
    const int64_t nb = ((int64_t)M * N + 255) / 256;
    hipLaunchKernelGGL(k_zsmall_ew, dim3((unsigned)nb), dim3(256), 0, st, M, N, a, (const cplx*)X, ldx, opx, b,
                       (const cplx*)Y, ldy, opy, c, mode, (cplx*)D, ldd);
    return hipGetLastError();
}

hipError_t launch_zcopy(int64_t M, int N, const void* src, int64_t lds, void* dst, int64_t ldd, hipStream_t st) {
    if (M <= 0 || N <= 0) return hipSuccess;
    const int64_t nb = (M * N + 255) / 256;
    hipLaunchKernelGGL(k_zcopy, dim3((unsigned)nb), dim3(256), 0, st, M, N, (const cplx*)src, lds, (cplx*)dst, ldd);
    return hipGetLastError();
}

}  // namespace tho
