// Chunked tall-skinny Householder QR (the intra-block QR of line 6 of
// Algorithm 1) and the explicit formation of Q (line 7), for gfx950.
//
// Structure.  The m x k matrix is split into `nchunk` row chunks, one
// workgroup each.  A workgroup walks its chunk in tiles of 256 rows and keeps
// a running k x k triangle R in LDS (a flat reduction tree inside the chunk):
//   tile 0:  plain Householder QR of the tile,          X_0 = H_0 [I; 0] R
//   tile t:  QR of [R; X_t] with structured reflectors   u_j = [e_j; y_j]
// Every tile stores its Householder vectors Y_t (into the output buffer, in
// place of the rows of Q they will become) and its compact-WY factor T_t
// (H_t = I - U_t T_t U_t^T), so Q can be formed later without refactoring.
// The chunk R factors are stacked into the matrix of the next level, which is
// reduced the same way until one chunk remains.
//
// Level 0 (the bottom n - k0 rows of A) is fused with the generalized
// Householder step of Algorithm 1: the tile loaded from A is updated to
// A + V Z on MFMA before factorization (line 4), and the chunk accumulates
// N_c = V_chunk^T Q_chunk, which gives W^T [0; Q_] = -sum_c N_c G_c without
// another pass over V (line 7).
//
// Register tile: 8 wavefronts x 32 rows; each wavefront keeps two 16 x KP
// row blocks in FP64 MFMA accumulator layout (see tho_device.h), so the
// column reductions of the Householder loop are shuffles across the four
// 16-lane groups plus one LDS exchange across wavefronts, and the tile is
// directly an MFMA operand for products that contract over rows.
#include "tho_device.h"
#include "tho_internal.h"

namespace tho {

namespace {

constexpr int NW = LEAF_WAVES;
constexpr int TB = LEAF_ROWS;
constexpr int RB = 2;  // 16-row blocks per wavefront

__device__ __forceinline__ int tile_row(int w, int rb, int l, int v) {
    return 32 * w + 16 * rb + drow(l, v);
}

template <int KP, int K0P>
struct LeafLds {
    static constexpr int LDT = KP + 1;
    static constexpr int STG = (K0P > 0) ? K0P * (KP + 2) : 0;
    static constexpr int total =
        2 * KP * LDT + 2 * TB + 2 * NW + 4 + 2 * NW * KP + KP + STG;
};

template <int KP, int K0P>
struct FormLds {
    static constexpr int LDT = KP + 1;
    static constexpr int total = KP * LDT + KP * LDT + K0P * KP;
};

}  // namespace

template <int KP, int K0P>
__global__ __launch_bounds__(512) void k_tsqr_leaf(TsqrLevel L) {
    constexpr int CT = KP / 16;
    constexpr int LDT = KP + 1;
    constexpr bool HASV = K0P > 0;
    constexpr int KS0 = (K0P > 0) ? K0P / 4 : 1;
    constexpr int MT0 = K0P / 16;
    constexpr int NTILE = MT0 * CT;
    constexpr int NTW = (NTILE > 0) ? (NTILE + NW - 1) / NW : 1;
    constexpr int SP = KP + 2;  // pitch of the N staging buffer

    extern __shared__ double sm[];
    double* Tl = sm;                    // KP x LDT: T of the current tile
    double* slot = Tl + KP * LDT;       // KP x LDT: running R of the chunk
    double* xcol = slot + KP * LDT;     // 2 x TB: pivot column (double buffered)
    double* red = xcol + 2 * TB;        // 2 x NW: partial norms
    double* alph = red + 2 * NW;        // 2 (+2): pivot of the plain tile
    double* part = alph + 4;            // 2 x NW x KP: partial dot products
    double* wcp = part + 2 * NW * KP;   // KP: dot products for the T recurrence
    double* stage = wcp + KP;           // level 0: Z (permuted) / N staging

    const int tid = threadIdx.x, l = tid & 63, w = tid >> 6, g = l >> 4, cl = l & 15;
    const int c = blockIdx.x;
    const int k = L.k;
    const int k0 = HASV ? L.k0 : 0;
    const int64_t cr0 = (int64_t)c * L.m / L.nchunk;
    const int64_t cr1 = (int64_t)(c + 1) * L.m / L.nchunk;
    const int ntiles = (int)((cr1 - cr0 + TB - 1) / TB);

    d4 nacc[NTW];
#pragma unroll
    for (int i = 0; i < NTW; i++) nacc[i] = d4zero();

    for (int t = 0; t < ntiles; t++) {
        const int64_t r0 = cr0 + (int64_t)t * TB;
        const int trows = (int)((cr1 - r0 < TB) ? (cr1 - r0) : TB);
        const bool plain = (t == 0);

        // ---- load the tile (rows r0.., in accumulator layout)
        d4 x[RB][CT];
#pragma unroll
        for (int rb = 0; rb < RB; rb++)
#pragma unroll
            for (int ct = 0; ct < CT; ct++)
#pragma unroll
                for (int v = 0; v < 4; v++) {
                    const int row = tile_row(w, rb, l, v), col = 16 * ct + cl;
                    x[rb][ct][v] = (row < trows && col < k) ? L.X[(r0 + row) * L.ldx + col] : 0.0;
                }
        for (int e = tid; e < KP * LDT; e += blockDim.x) Tl[e] = 0.0;

        // ---- line 4 of Algorithm 1 on these rows: A <- A + V Z  (MFMA)
        if (HASV && k0 > 0) {
            __syncthreads();  // previous use of the staging area is over
            for (int e = tid; e < KS0 * CT * 64; e += blockDim.x) {
                const int ll = e & 63, sc = e >> 6, s = sc / CT, ct = sc % CT;
                stage[e] = L.Z[((ll >> 4) * KS0 + s) * KP + 16 * ct + (ll & 15)];
            }
            __syncthreads();
#pragma unroll
            for (int rb = 0; rb < RB; rb++) {
                const int vr = 32 * w + 16 * rb + cl;  // A-operand row of this lane
                const bool vok = vr < trows;
                const double* vp = L.V + (r0 + vr) * L.ldv + g * KS0;
                double a[KS0];
#pragma unroll
                for (int s = 0; s < KS0; s++) a[s] = (vok && g * KS0 + s < k0) ? vp[s] : 0.0;
#pragma unroll
                for (int s = 0; s < KS0; s++)
#pragma unroll
                    for (int ct = 0; ct < CT; ct++)
                        x[rb][ct] = mfma(a[s], stage[(s * CT + ct) * 64 + l], x[rb][ct]);
            }
        }

        // ---- Householder QR of the tile (plain) or of [R; tile] (structured)
        double tau_prev = 0.0, beta_prev = 0.0, wl_prev = 0.0;
        for (int j = 0; j < k; j++) {
            const int pb = j & 1, ctj = j >> 4, clj = j & 15;
            double xj[RB][4];
#pragma unroll
            for (int rb = 0; rb < RB; rb++)
#pragma unroll
                for (int v = 0; v < 4; v++) {
                    double vv = 0.0;
#pragma unroll
                    for (int ct = 0; ct < CT; ct++)
                        if (ct == ctj) vv = x[rb][ct][v];
                    xj[rb][v] = vv;
                }
            double ss = 0.0;
            if (cl == clj) {
#pragma unroll
                for (int rb = 0; rb < RB; rb++)
#pragma unroll
                    for (int v = 0; v < 4; v++) {
                        const int row = tile_row(w, rb, l, v);
                        const double vv = xj[rb][v];
                        if (!plain || row > j) ss += vv * vv;
                        xcol[pb * TB + row] = vv;
                        if (plain && row == j) alph[pb] = vv;
                    }
            }
            ss = sum_groups(ss);
            if (l == clj) red[pb * NW + w] = ss;
            __syncthreads();

            double sig2 = 0.0;
#pragma unroll
            for (int ww = 0; ww < NW; ww++) sig2 += red[pb * NW + ww];
            const double alpha = plain ? alph[pb] : slot[j * LDT + j];
            double beta = alpha, tau = 0.0, scale = 0.0;
            if (sig2 != 0.0) {
                const double nrm = sqrt(alpha * alpha + sig2);
                beta = (alpha < 0.0) ? nrm : -nrm;
                tau = (beta - alpha) / beta;
                scale = 1.0 / (alpha - beta);
            }
            double u[RB][4];
#pragma unroll
            for (int rb = 0; rb < RB; rb++)
#pragma unroll
                for (int v = 0; v < 4; v++) {
                    const int row = tile_row(w, rb, l, v);
                    const double xr = xcol[pb * TB + row];
                    u[rb][v] = plain ? ((row > j) ? xr * scale : ((row == j) ? 1.0 : 0.0)) : xr * scale;
                }
            // dot products of u with every column (trailing ones: update;
            // leading ones: the T recurrence)
#pragma unroll
            for (int ct = 0; ct < CT; ct++) {
                double s = 0.0;
#pragma unroll
                for (int rb = 0; rb < RB; rb++)
#pragma unroll
                    for (int v = 0; v < 4; v++) s += u[rb][v] * x[rb][ct][v];
                s = sum_groups(s);
                if (g == 0) part[(pb * NW + w) * KP + 16 * ct + cl] = s;
            }
            // deferred update of slot row j-1 (its readers are past barrier 1)
            if (!plain && j > 0 && w == 0) {
                if (l > j - 1 && l < k) slot[(j - 1) * LDT + l] -= tau_prev * wl_prev;
                if (l == j - 1) slot[(j - 1) * LDT + (j - 1)] = beta_prev;
            }
            __syncthreads();

            double wl = 0.0;
            if (l < KP) {
#pragma unroll
                for (int ww = 0; ww < NW; ww++) wl += part[(pb * NW + ww) * KP + l];
                if (!plain) wl += slot[j * LDT + l];
            }
            double wv[CT];
#pragma unroll
            for (int ct = 0; ct < CT; ct++) wv[ct] = __shfl(wl, 16 * ct + cl);
#pragma unroll
            for (int ct = 0; ct < CT; ct++) {
                const int col = 16 * ct + cl;
                const double coef = (col > j && col < k) ? tau * wv[ct] : 0.0;
#pragma unroll
                for (int rb = 0; rb < RB; rb++)
#pragma unroll
                    for (int v = 0; v < 4; v++) x[rb][ct][v] -= coef * u[rb][v];
            }
            // column j becomes the Householder vector (and beta on the pivot)
#pragma unroll
            for (int ct = 0; ct < CT; ct++) {
                if (ct == ctj && cl == clj) {
#pragma unroll
                    for (int rb = 0; rb < RB; rb++)
#pragma unroll
                        for (int v = 0; v < 4; v++) {
                            const int row = tile_row(w, rb, l, v);
                            if (!plain || row > j) x[rb][ct][v] = u[rb][v];
                            else if (row == j) x[rb][ct][v] = beta;
                        }
                }
            }
            // T(0:j, j) = -tau T(0:j, 0:j) (U(:,0:j)^T u_j),  T(j, j) = tau
            if (w == NW - 1) {
                if (l < KP) wcp[l] = wl;
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                if (l < j) {
                    double s = 0.0;
                    for (int p = l; p < j; p++) s += Tl[l * LDT + p] * wcp[p];
                    Tl[l * LDT + j] = -tau * s;
                }
                if (l == j) Tl[j * LDT + j] = tau;
            }
            tau_prev = tau;
            beta_prev = beta;
            wl_prev = wl;
        }
        if (!plain && w == 0 && k > 0 && l == k - 1) slot[(k - 1) * LDT + (k - 1)] = beta_prev;
        __syncthreads();

        if (plain) {
            // R -> slot; registers -> unit lower trapezoidal Y
#pragma unroll
            for (int rb = 0; rb < RB; rb++)
#pragma unroll
                for (int ct = 0; ct < CT; ct++)
#pragma unroll
                    for (int v = 0; v < 4; v++) {
                        const int row = tile_row(w, rb, l, v), col = 16 * ct + cl;
                        if (row < KP && col < KP) {
                            const double xv = x[rb][ct][v];
                            slot[row * LDT + col] = (col >= row && row < k && col < k) ? xv : 0.0;
                            if (col > row) x[rb][ct][v] = 0.0;
                            else if (col == row) x[rb][ct][v] = (row < k) ? 1.0 : 0.0;
                        }
                    }
        }
        // store Y_t and T_t
#pragma unroll
        for (int rb = 0; rb < RB; rb++)
#pragma unroll
            for (int ct = 0; ct < CT; ct++)
#pragma unroll
                for (int v = 0; v < 4; v++) {
                    const int row = tile_row(w, rb, l, v), col = 16 * ct + cl;
                    if (row < trows && col < k) L.Y[(r0 + row) * L.ldy + col] = x[rb][ct][v];
                }
        {
            const int64_t ti = (int64_t)c * L.maxtiles + t;
            double* Tg = L.Tt + ti * KP * KP;
            for (int e = tid; e < KP * KP; e += blockDim.x) Tg[e] = Tl[(e / KP) * LDT + (e % KP)];
        }
        __syncthreads();

        // ---- level 0: N_c <- V^T Q of the chunk so far
        if (HASV && k0 > 0) {
            d4 bacc[NTW];
#pragma unroll
            for (int i = 0; i < NTW; i++) bacc[i] = d4zero();
            for (int s = 0; s < TB / 4; s++) {
                const int row = 4 * s + g;
                const bool ok = row < trows;
#pragma unroll
                for (int i = 0; i < NTW; i++) {
                    const int id = w + NW * i;
                    if (id < NTILE) {
                        const int mi = id / CT, nj = id % CT;
                        const int vc = 16 * mi + cl, yc = 16 * nj + cl;
                        const double a = (ok && vc < k0) ? L.V[(r0 + row) * L.ldv + vc] : 0.0;
                        const double b = (ok && yc < k) ? L.Y[(r0 + row) * L.ldy + yc] : 0.0;
                        bacc[i] = mfma(a, b, bacc[i]);
                    }
                }
            }
            // stage (N + B) (or B for the plain tile), then D = stage * T
#pragma unroll
            for (int i = 0; i < NTW; i++) {
                const int id = w + NW * i;
                if (id < NTILE) {
                    const int mi = id / CT, nj = id % CT;
#pragma unroll
                    for (int v = 0; v < 4; v++)
                        stage[(16 * mi + drow(l, v)) * SP + 16 * nj + cl] =
                            bacc[i][v] + (plain ? 0.0 : nacc[i][v]);
                }
            }
            __syncthreads();
            d4 dacc[NTW];
#pragma unroll
            for (int i = 0; i < NTW; i++) dacc[i] = d4zero();
#pragma unroll
            for (int s = 0; s < KP / 4; s++)
#pragma unroll
                for (int i = 0; i < NTW; i++) {
                    const int id = w + NW * i;
                    if (id < NTILE) {
                        const int mi = id / CT, nj = id % CT;
                        const double a = stage[(16 * mi + cl) * SP + 4 * s + g];
                        const double b = Tl[(4 * s + g) * LDT + 16 * nj + cl];
                        dacc[i] = mfma(a, b, dacc[i]);
                    }
                }
            if (!plain) {
#pragma unroll
                for (int i = 0; i < NTW; i++) nacc[i] -= dacc[i];
            } else {
                // N = V_0[0:k]^T - (B_0 T_0) L_0^T with L_0 = Y_0[0:k, 0:k]
                __syncthreads();
#pragma unroll
                for (int i = 0; i < NTW; i++) {
                    const int id = w + NW * i;
                    if (id < NTILE) {
                        const int mi = id / CT, nj = id % CT;
#pragma unroll
                        for (int v = 0; v < 4; v++)
                            stage[(16 * mi + drow(l, v)) * SP + 16 * nj + cl] = dacc[i][v];
                    }
                }
                __syncthreads();
                d4 eacc[NTW];
#pragma unroll
                for (int i = 0; i < NTW; i++) eacc[i] = d4zero();
#pragma unroll
                for (int s = 0; s < KP / 4; s++)
#pragma unroll
                    for (int i = 0; i < NTW; i++) {
                        const int id = w + NW * i;
                        if (id < NTILE) {
                            const int mi = id / CT, nj = id % CT;
                            const double a = stage[(16 * mi + cl) * SP + 4 * s + g];
                            const int lr = 16 * nj + cl, lc = 4 * s + g;
                            const double b = (lr < k && lc < k) ? L.Y[(r0 + lr) * L.ldy + lc] : 0.0;
                            eacc[i] = mfma(a, b, eacc[i]);
                        }
                    }
#pragma unroll
                for (int i = 0; i < NTW; i++) {
                    const int id = w + NW * i;
                    if (id < NTILE) {
                        const int mi = id / CT, nj = id % CT;
#pragma unroll
                        for (int v = 0; v < 4; v++) {
                            const int r = 16 * mi + drow(l, v), cc = 16 * nj + cl;
                            const double vt = (r < k0 && cc < k) ? L.V[(r0 + cc) * L.ldv + r] : 0.0;
                            nacc[i][v] = vt - eacc[i][v];
                        }
                    }
                }
            }
        }
    }

    // ---- chunk outputs: R_c into the next level, N_c
    for (int e = tid; e < k * KP; e += blockDim.x) {
        const int i = e / KP, jj = e % KP;
        L.Rnext[((int64_t)c * k + i) * L.ldrn + jj] = (jj < k && jj >= i) ? slot[i * LDT + jj] : 0.0;
    }
    if (HASV && k0 > 0) {
        double* Nout = L.Nc + (int64_t)c * K0P * KP;
#pragma unroll
        for (int i = 0; i < NTW; i++) {
            const int id = w + NW * i;
            if (id < NTILE) {
                const int mi = id / CT, nj = id % CT;
#pragma unroll
                for (int v = 0; v < 4; v++)
                    Nout[(16 * mi + drow(l, v)) * KP + 16 * nj + cl] = nacc[i][v];
            }
        }
    }
}

// Form the explicit Q of one level from the stored Householder vectors:
// chunk c's rows of Q are Q_chunk G_c, with G_c read from the formed level
// above (or the phase signs at the top).  Tiles are visited last to first;
// C carries G_c down the flat tree:
//   structured tile t:  K = T_t C,                rows = -Y_t K,  C <- C - K
//   plain tile 0:       K = T_0 (Y_0[0:k]^T C),   rows = [C; 0] - Y_0 K
// Level 0 adds V N (line 7 of Algorithm 1: Q_low = Q_ + V_low N).
// Output rows overwrite the Householder vectors in place.
template <int KP, int K0P>
__global__ __launch_bounds__(512) void k_tsqr_form(TsqrLevel L) {
    constexpr int CT = KP / 16;
    constexpr int LDT = KP + 1;
    constexpr bool HASV = K0P > 0;
    constexpr int KS0 = (K0P > 0) ? K0P / 4 : 1;
    constexpr int KSK = KP / 4;
    constexpr int NTK = CT * CT;
    constexpr int NTKW = (NTK + NW - 1) / NW;

    extern __shared__ double sm[];
    double* Cm = sm;              // KP x LDT
    double* Kp = Cm + KP * LDT;   // KP x LDT region: E (plain) then -K permuted
    double* Np = Kp + KP * LDT;   // K0P * KP: N permuted

    const int tid = threadIdx.x, l = tid & 63, w = tid >> 6, g = l >> 4, cl = l & 15;
    const int c = blockIdx.x;
    const int k = L.k;
    const int k0 = HASV ? L.k0 : 0;
    const int64_t cr0 = (int64_t)c * L.m / L.nchunk;
    const int64_t cr1 = (int64_t)(c + 1) * L.m / L.nchunk;
    const int ntiles = (int)((cr1 - cr0 + TB - 1) / TB);

    {
        const double* G = L.Gin + (int64_t)c * L.gstride * L.ldg;
        for (int e = tid; e < KP * KP; e += blockDim.x) {
            const int i = e / KP, jj = e % KP;
            Cm[i * LDT + jj] = (i < k && jj < k) ? G[(int64_t)i * L.ldg + jj] : 0.0;
        }
        if (HASV && k0 > 0) {
            for (int e = tid; e < KS0 * CT * 64; e += blockDim.x) {
                const int ll = e & 63, sc = e >> 6, s = sc / CT, ct = sc % CT;
                Np[e] = L.Nglob[((ll >> 4) * KS0 + s) * KP + 16 * ct + (ll & 15)];
            }
        }
    }
    __syncthreads();

    for (int t = ntiles - 1; t >= 0; t--) {
        const int64_t r0 = cr0 + (int64_t)t * TB;
        const int trows = (int)((cr1 - r0 < TB) ? (cr1 - r0) : TB);
        const bool plain = (t == 0);
        const double* Tg = L.Tt + ((int64_t)c * L.maxtiles + t) * KP * KP;

        const double* src = Cm;
        if (plain) {
            d4 e[NTKW];
#pragma unroll
            for (int i = 0; i < NTKW; i++) e[i] = d4zero();
#pragma unroll
            for (int s = 0; s < KSK; s++)
#pragma unroll
                for (int i = 0; i < NTKW; i++) {
                    const int id = w + NW * i;
                    if (id < NTK) {
                        const int mi = id / CT, nj = id % CT;
                        const int yr = 4 * s + g, yc = 16 * mi + cl;
                        const double a = (yr < k && yc < k) ? L.Y[(r0 + yr) * L.ldy + yc] : 0.0;
                        e[i] = mfma(a, Cm[(4 * s + g) * LDT + 16 * nj + cl], e[i]);
                    }
                }
#pragma unroll
            for (int i = 0; i < NTKW; i++) {
                const int id = w + NW * i;
                if (id < NTK) {
                    const int mi = id / CT, nj = id % CT;
#pragma unroll
                    for (int v = 0; v < 4; v++) Kp[(16 * mi + drow(l, v)) * LDT + 16 * nj + cl] = e[i][v];
                }
            }
            __syncthreads();
            src = Kp;
        }
        d4 kk[NTKW];
#pragma unroll
        for (int i = 0; i < NTKW; i++) kk[i] = d4zero();
#pragma unroll
        for (int s = 0; s < KSK; s++)
#pragma unroll
            for (int i = 0; i < NTKW; i++) {
                const int id = w + NW * i;
                if (id < NTK) {
                    const int mi = id / CT, nj = id % CT;
                    const double a = Tg[(16 * mi + cl) * KP + 4 * s + g];
                    kk[i] = mfma(a, src[(4 * s + g) * LDT + 16 * nj + cl], kk[i]);
                }
            }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NTKW; i++) {
            const int id = w + NW * i;
            if (id < NTK) {
                const int mi = id / CT, nj = id % CT;
#pragma unroll
                for (int v = 0; v < 4; v++) {
                    const int r = 16 * mi + drow(l, v), cc = 16 * nj + cl;
                    const int gg = r / KSK, s = r % KSK;
                    Kp[(s * CT + (cc >> 4)) * 64 + 16 * gg + (cc & 15)] = -kk[i][v];
                    if (!plain) Cm[r * LDT + cc] -= kk[i][v];
                }
            }
        }
        __syncthreads();

        d4 acc[RB][CT];
#pragma unroll
        for (int rb = 0; rb < RB; rb++)
#pragma unroll
            for (int ct = 0; ct < CT; ct++)
#pragma unroll
                for (int v = 0; v < 4; v++) {
                    const int row = tile_row(w, rb, l, v), col = 16 * ct + cl;
                    acc[rb][ct][v] = (plain && row < k && col < k) ? Cm[row * LDT + col] : 0.0;
                }
#pragma unroll
        for (int rb = 0; rb < RB; rb++) {
            const int yr = 32 * w + 16 * rb + cl;
            const bool ok = yr < trows;
            {
                const double* yp = L.Y + (r0 + yr) * L.ldy + g * KSK;
                double a[KSK];
#pragma unroll
                for (int s = 0; s < KSK; s++) a[s] = (ok && g * KSK + s < k) ? yp[s] : 0.0;
#pragma unroll
                for (int s = 0; s < KSK; s++)
#pragma unroll
                    for (int ct = 0; ct < CT; ct++)
                        acc[rb][ct] = mfma(a[s], Kp[(s * CT + ct) * 64 + l], acc[rb][ct]);
            }
            if (HASV && k0 > 0) {
                const double* vp = L.V + (r0 + yr) * L.ldv + g * KS0;
                double a[KS0];
#pragma unroll
                for (int s = 0; s < KS0; s++) a[s] = (ok && g * KS0 + s < k0) ? vp[s] : 0.0;
#pragma unroll
                for (int s = 0; s < KS0; s++)
#pragma unroll
                    for (int ct = 0; ct < CT; ct++)
                        acc[rb][ct] = mfma(a[s], Np[(s * CT + ct) * 64 + l], acc[rb][ct]);
            }
        }
#pragma unroll
        for (int rb = 0; rb < RB; rb++)
#pragma unroll
            for (int ct = 0; ct < CT; ct++)
#pragma unroll
                for (int v = 0; v < 4; v++) {
                    const int row = tile_row(w, rb, l, v), col = 16 * ct + cl;
                    if (row < trows && col < k) L.Y[(r0 + row) * L.ldy + col] = acc[rb][ct][v];
                }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- launchers

template <int KP, int K0P>
static hipError_t leaf_t(const TsqrLevel& L, hipStream_t st) {
    const size_t shm = LeafLds<KP, K0P>::total * sizeof(double);
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void*)k_tsqr_leaf<KP, K0P>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL((k_tsqr_leaf<KP, K0P>), dim3(L.nchunk), dim3(NW * 64), shm, st, L);
    return hipGetLastError();
}

template <int KP, int K0P>
static hipError_t form_t(const TsqrLevel& L, hipStream_t st) {
    const size_t shm = FormLds<KP, K0P>::total * sizeof(double);
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void*)k_tsqr_form<KP, K0P>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL((k_tsqr_form<KP, K0P>), dim3(L.nchunk), dim3(NW * 64), shm, st, L);
    return hipGetLastError();
}

#define TSQR_DISPATCH(FN)                                  \
    switch (kp * 1000 + k0p) {                             \
        case 16000: return FN<16, 0>(L, st);               \
        case 16016: return FN<16, 16>(L, st);              \
        case 16032: return FN<16, 32>(L, st);              \
        case 16064: return FN<16, 64>(L, st);              \
        case 16128: return FN<16, 128>(L, st);             \
        case 32000: return FN<32, 0>(L, st);               \
        case 32016: return FN<32, 16>(L, st);              \
        case 32032: return FN<32, 32>(L, st);              \
        case 32064: return FN<32, 64>(L, st);              \
        case 32128: return FN<32, 128>(L, st);             \
        case 64000: return FN<64, 0>(L, st);               \
        case 64016: return FN<64, 16>(L, st);              \
        case 64032: return FN<64, 32>(L, st);              \
        case 64064: return FN<64, 64>(L, st);              \
        case 64128: return FN<64, 128>(L, st);             \
        default: return hipErrorInvalidValue;              \
    }

hipError_t launch_tsqr_leaf(int kp, int k0p, const TsqrLevel& L, hipStream_t st) {
    TSQR_DISPATCH(leaf_t)
}

hipError_t launch_tsqr_form(int kp, int k0p, const TsqrLevel& L, hipStream_t st) {
    TSQR_DISPATCH(form_t)
}

}  // namespace tho
