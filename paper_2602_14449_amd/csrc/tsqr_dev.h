// Chunked tall-skinny Householder QR (the QR of the bottom block in
// Algorithm 1) and the explicit formation of Q, for gfx950.
//
// Structure.  The m x k matrix is split into `nchunk` row chunks, one
// workgroup each.  A workgroup walks its chunk in tiles of 128 or 256 rows and keeps
// a running k x k triangle R in LDS (a flat reduction tree inside the chunk):
//   tile 0:  plain Householder QR of the tile,          X_0 = H_0 [I; 0] R
//   tile t:  QR of [R; X_t] with structured reflectors   u_j = [e_j; y_j]
// Every tile stores its Householder vectors Y_t (into the output buffer, in
// place of the rows of Q they will become) and its compact-WY factor T_t
// (H_t = I - U_t T_t U_t^T), so Q can be formed later without refactoring.
// The chunk R factors are stacked into the matrix of the next level, which is
// reduced the same way until one chunk remains.  Q is formed top-down: the
// upper levels chunk by chunk (form_chunk), level 0 in two passes (the k x k
// recurrence per chunk, then every tile on its own; see kchain_chunk).
//
// Level 0 (the bottom n - k0 rows of A) is fused with the generalized
// Householder step of Algorithm 1: the tile loaded from A is updated to
// A + V Z on MFMA before factorization (the update of A), and the chunk accumulates
// N_c = V_chunk^T Q_chunk, which gives W^T [0; Q_] = -sum_c N_c G_c without
// another pass over V (formation of Q).
//
// Register tile: 4 wavefronts x 32 or 64 rows; each wavefront keeps two or
// four 16 x KP row blocks in FP64 MFMA accumulator layout (tho_device.h), so the
// column reductions of the Householder loop are shuffles across the four
// 16-lane groups plus one LDS exchange across wavefronts, and the tile is
// directly an MFMA operand for products that contract over rows.
#pragma once

#include "tho_device.h"
#include "tho_internal.h"
#include "tho_lowp.h"

namespace tho {

#ifdef THO_PHASE_TIMING
static __device__ long long g_phase_ts[4096];
#define PHASE_TS(t, ph) \
    do { if (blockIdx.x == 0 && threadIdx.x == 0 && (t) < 64) g_phase_ts[(t) * 8 + (ph)] = clock64(); } while (0)
#else
#define PHASE_TS(t, ph) do {} while (0)
#endif

namespace {

constexpr int NW = LEAF_WAVES;     // wavefronts per workgroup

// Tile geometry per column count: the register tile is RB 16-row blocks per
// wavefront (KP = 64: 2 blocks, so that a wavefront fits in 256 registers
// and two workgroups share a compute unit; narrower: 4 blocks).
template <int KP, int RBO = 0, int NWT = NW>
struct Geo {
    static constexpr int RB = RBO ? RBO : ((KP >= 64) ? 2 : 4);  // 16-row blocks per wavefront
    static constexpr int RPW = 16 * RB;            // rows per wavefront
    static constexpr int TB = NWT * RPW;           // rows per tile (NWT wavefronts)
};

// Lane id the compiler cannot treat as loop invariant: per-lane address
// offsets derived from it are recomputed in each phase instead of being
// hoisted and kept live across the Householder loop (register pressure).
__device__ __forceinline__ int opaque_lane() {
    int x = threadIdx.x & 63;
    asm volatile("" : "+v"(x));
    return x;
}

template <int RPW>
__device__ __forceinline__ int tile_row(int w, int rb, int l, int v) {
    return RPW * w + 16 * rb + drow(l, v);
}

template <int KP, int RBO = 0, int NWT = NW>
struct LeafLds {
    static constexpr int LDT = KP + 1;
    static constexpr int total = 2 * KP * LDT + Geo<KP, RBO, NWT>::TB + 2 * KP + 2 * NWT * KP + KP;
};

template <int KP>
struct FormLds {
    static constexpr int LDT = KP + 1;
    static constexpr int total = KP * LDT + KP * LDT;
};

// State handed from one Householder column to the next.
struct HhCarry {
    double beta_prev;  // beta of the previous reflector
    double rnew;       // structured: my entry of the previous pivot row after its reflector
    double myscale;    // 1 / (alpha - beta) of the reflector of column `lane` (0 until then)
};

// Columns 16 CTJ .. min(16 CTJ + 16, k) - 1 of the Householder QR of the
// register tile (see householder_tile).  With the pivot column block a
// compile-time constant, the block selections are static: only the pivot
// block's lanes take a lane mask, blocks left of it (Householder vectors) are
// not updated, and no scalar branches are spent on the block index.
template <int KP, bool PLAIN, int RBO, int NWT, int CTJ>
__device__ __forceinline__ void householder_block(d4 (&x)[(Geo<KP, RBO>::RB)][KP / 16], int k, int w,
                                                  double* xcol, double* prow, double* part, double* slot,
                                                  double* Gm, double* taus, HhCarry& cy) {
    constexpr int RB = Geo<KP, RBO>::RB, RPW = Geo<KP, RBO>::RPW;
    constexpr int CT = KP / 16;
    constexpr int LDT = KP + 1;
    const int l = opaque_lane(), g = l >> 4, cl = l & 15;
    double* xw = xcol + RPW * w;  // this wavefront's pivot column, lane-group order
    const int jend = (16 * CTJ + 16 < k) ? 16 * CTJ + 16 : k;
    for (int j = 16 * CTJ; j < jend; j++) {
        const int pb = j & 1, clj = j & 15;
        if (cl == clj) {
#pragma unroll
            for (int rb = 0; rb < RB; rb++)
#pragma unroll
                for (int v = 0; v < 4; v++) xw[rb * 16 + g * 4 + v] = x[rb][CTJ][v];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        double xs[RB][4];  // pivot-column value on my sub rows, 0 elsewhere
#pragma unroll
        for (int rb = 0; rb < RB; rb++)
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const double xv = xw[rb * 16 + g * 4 + v];
                xs[rb][v] = (!PLAIN || tile_row<RPW>(w, rb, l, v) > j) ? xv : 0.0;
            }
        {
            // CT independent dot products, interleaved so that the FMA chains
            // and the cross-lane reductions pipeline (blocks left of the
            // pivot give the Gram of the Householder vectors for T)
            double sc[CT];
#pragma unroll
            for (int ct = 0; ct < CT; ct++) sc[ct] = 0.0;
#pragma unroll
            for (int rb = 0; rb < RB; rb++)
#pragma unroll
                for (int v = 0; v < 4; v++)
#pragma unroll
                    for (int ct = 0; ct < CT; ct++) sc[ct] += xs[rb][v] * x[rb][ct][v];
            const double tot = col_sums<CT>(sc);  // valid in lanes l < KP
            if (l < KP) part[(pb * NWT + w) * KP + l] = tot;
        }
        if (PLAIN && w == j / RPW) {
            // publish the pivot row (row j of the tile)
#pragma unroll
            for (int rb = 0; rb < RB; rb++)
#pragma unroll
                for (int v = 0; v < 4; v++)
                    if (tile_row<RPW>(w, rb, l, v) == j) {
#pragma unroll
                        for (int ct = 0; ct < CT; ct++) prow[pb * KP + 16 * ct + cl] = x[rb][ct][v];
                    }
        }
        __syncthreads();

        // row j-1 of the slot after its reflector (every reader of the old
        // row is past the barrier); plain stores, computed last column
        if (!PLAIN && j > 0 && w == 0) {
            if (l > j - 1 && l < k) slot[(j - 1) * LDT + l] = cy.rnew;
            if (l == j - 1) slot[(j - 1) * LDT + (j - 1)] = cy.beta_prev;
        }
        double dl = 0.0, pl = 0.0;
        if (l < KP) {
            double pp[NWT];
#pragma unroll
            for (int ww = 0; ww < NWT; ww++) pp[ww] = part[(pb * NWT + ww) * KP + l];
            pl = PLAIN ? prow[pb * KP + l] : slot[j * LDT + l];
#pragma unroll
            for (int ww = 0; ww < NWT; ww++) dl += pp[ww];
        }
        const double sig2 = bcast(dl, j);
        const double alpha = bcast(pl, j);
        double beta = alpha, tau = 0.0, scale = 0.0;
        if (sig2 != 0.0) {
            // beta = -sign(alpha) sqrt(alpha^2 + sigma^2) from the hardware
            // reciprocal square root r (two Newton steps), then one Newton
            // step for the root; tau = (beta - alpha) / beta = 1 + |alpha| r
            // needs no division, and the reflector's scale 1 / (alpha - beta)
            // is the hardware reciprocal with two Newton steps.  s is a
            // normal number over the documented input range.
            const double s2 = fma(alpha, alpha, sig2);
            double r = __builtin_amdgcn_rsq(s2);
            r = fma(0.5 * r, fma(-s2 * r, r, 1.0), r);
            r = fma(0.5 * r, fma(-s2 * r, r, 1.0), r);
            double nrm = s2 * r;
            nrm = fma(0.5 * r, fma(-nrm, nrm, s2), nrm);
            beta = (alpha < 0.0) ? nrm : -nrm;
            tau = fma(fabs(alpha), r, 1.0);
            const double amb = alpha - beta;
            double q = __builtin_amdgcn_rcp(amb);
            q = fma(q, fma(-amb, q, 1.0), q);
            q = fma(q, fma(-amb, q, 1.0), q);
            scale = q;
        }
        // w_c = u^T x_c for the trailing columns; for c < j, times the scale
        // of column c (still unscaled in the registers), u_c^T u_j for T
        const double wl = pl + scale * dl;
        if (!PLAIN) cy.rnew = pl - tau * wl;
        if (w == 0) {
            if (l < j) Gm[j * LDT + l] = wl * cy.myscale;
            if (l == 0) taus[j] = tau;
        }
        if (l == j) cy.myscale = scale;
        double wv[4];
        gather_cols(wl, wv);
        // rank-1 update of the columns right of j; padding columns (>= k)
        // stay zero by themselves, as their pivot-row entries and dot
        // products are zero
        double u[RB][4];  // plain: the reflector on my rows
        if (PLAIN) {
#pragma unroll
            for (int rb = 0; rb < RB; rb++)
#pragma unroll
                for (int v = 0; v < 4; v++)
                    u[rb][v] = (tile_row<RPW>(w, rb, l, v) == j) ? 1.0 : xs[rb][v] * scale;
        }
        const double ts = PLAIN ? tau : tau * scale;
#pragma unroll
        for (int ct = CTJ; ct < CT; ct++) {
            const double cw = ts * wv[ct];
            const double coef = (ct > CTJ || cl > clj) ? cw : 0.0;
#pragma unroll
            for (int rb = 0; rb < RB; rb++)
#pragma unroll
                for (int v = 0; v < 4; v++) x[rb][ct][v] -= coef * (PLAIN ? u[rb][v] : xs[rb][v]);
        }
        // plain: beta on the pivot (the sub-column keeps its unscaled values)
        if (PLAIN && cl == clj) {
#pragma unroll
            for (int rb = 0; rb < RB; rb++)
#pragma unroll
                for (int v = 0; v < 4; v++)
                    if (tile_row<RPW>(w, rb, l, v) == j) x[rb][CTJ][v] = beta;
        }
        cy.beta_prev = beta;
    }
}

// Householder QR of the register tile x (PLAIN: the tile alone; otherwise
// [slot; tile] with the running triangle in `slot`).  One cross-wavefront
// exchange per column: every wavefront reduces, over its "sub" rows (below
// the pivot), the dot products d_c of the unscaled pivot column with every
// column c.  With the pivot-row values p_c and the reflector
// u = [1; x_sub / (alpha - beta)]:
//   sigma^2 = d_j,   w_c = u^T x_c = p_c + d_c / (alpha - beta),
// and for c < j, w_c (times the scale of column c) = u_c^T u_j feeds the T
// recurrence (Gm).  The Householder vectors stay unscaled in the registers
// during the loop and are scaled once at the end.  Returns beta of the last
// column; for a structured tile the caller stores it into slot(k-1, k-1)
// after the next workgroup barrier (other wavefronts read that entry as the
// pivot of the last column until then).
template <int KP, bool PLAIN, int RBO, int NWT = NW>
__device__ __forceinline__ double householder_tile(d4 (&x)[(Geo<KP, RBO>::RB)][KP / 16], int k, int w, double* xcol,
                                                 double* prow, double* part, double* slot, double* Gm,
                                                 double* taus) {
    constexpr int RB = Geo<KP, RBO>::RB, RPW = Geo<KP, RBO>::RPW;
    constexpr int CT = KP / 16;
    HhCarry cy = {0.0, 0.0, 0.0};
    householder_block<KP, PLAIN, RBO, NWT, 0>(x, k, w, xcol, prow, part, slot, Gm, taus, cy);
    if constexpr (CT > 1) householder_block<KP, PLAIN, RBO, NWT, 1>(x, k, w, xcol, prow, part, slot, Gm, taus, cy);
    if constexpr (CT > 2) householder_block<KP, PLAIN, RBO, NWT, 2>(x, k, w, xcol, prow, part, slot, Gm, taus, cy);
    if constexpr (CT > 3) householder_block<KP, PLAIN, RBO, NWT, 3>(x, k, w, xcol, prow, part, slot, Gm, taus, cy);
    // scale the Householder vectors: column c = 16 ct + l % 16 by its
    // 1 / (alpha - beta) (0 for padding columns and tau = 0 columns, whose
    // sub-columns are zero); the plain tile's rows <= c hold R
    double sv[4];
    gather_cols(cy.myscale, sv);
    const int l = opaque_lane(), cl = l & 15;
#pragma unroll
    for (int rb = 0; rb < RB; rb++)
#pragma unroll
        for (int ct = 0; ct < CT; ct++)
#pragma unroll
            for (int v = 0; v < 4; v++) {
                if (PLAIN) {
                    if (tile_row<RPW>(w, rb, l, v) > 16 * ct + cl) x[rb][ct][v] *= sv[ct];
                } else {
                    x[rb][ct][v] *= sv[ct];
                }
            }
    return cy.beta_prev;
}

// T factor of the tile in TG (see leaf_chunk).  Diagonal 16 x 16 blocks by
// the column recurrence (four lanes per row, entries p = 16 b + lane + 4 q in
// registers, quad reductions), then merges on MFMA.  TG holds only finite
// values (it is cleared once per chunk), so no load needs a mask.  Ends
// before a workgroup barrier of the caller.
template <int KP>
__device__ __forceinline__ void tile_t_factor(double* TG, const double* taus, int k, int w) {
    constexpr int CT = KP / 16;
    constexpr int LDT = KP + 1;
    // thread index the compiler cannot hoist: addresses derived from it are
    // recomputed here instead of being kept live across the tile loop
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    if (w < CT) {
        const int tq = tid & 3, ti = tid >> 2;  // row ti = 16 w + (lane / 4) of block w
        const int p0 = 16 * w + tq;             // entries p = p0 + 4 q
        double Tr[4];
#pragma unroll
        for (int q = 0; q < 4; q++) Tr[q] = (p0 + 4 * q == ti && ti < k) ? taus[ti] : 0.0;
        const int jend = (16 * w + 16 < k) ? 16 * w + 16 : k;
        for (int j = 16 * w + 1; j < jend; j++) {
            double sr = 0.0;
#pragma unroll
            for (int q = 0; q < 4; q++) sr += Tr[q] * TG[j * LDT + p0 + 4 * q];
            sr = sum_quad(sr);
            const int qj = (j - 16 * w) >> 2;
            const double v = -taus[j] * sr;
            const bool mine = j > ti && tq == (j & 3);
#pragma unroll
            for (int q = 0; q < 4; q++)
                if (q == qj && mine) Tr[q] = v;
        }
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const int p = p0 + 4 * q;
            if (p >= ti) TG[ti * LDT + p] = Tr[q];
        }
    }
    if constexpr (CT >= 2) {
        const int l = tid & 63, g = l >> 4, cl = l & 15;
        __syncthreads();
        // pairs of 16: blocks (a, b) = (2 w, 2 w + 1)
        if (w < CT / 2) {
            const int a = 2 * w, b = 2 * w + 1;
            d4 x = d4zero(), y = d4zero();
#pragma unroll
            for (int s = 0; s < 4; s++) {  // X = G_ab T_b, K index 4 s + g
                const int kk = 4 * s + g;
                const double ga = TG[(16 * b + kk) * LDT + 16 * a + cl];
                const double tb = (kk <= cl) ? TG[(16 * b + kk) * LDT + 16 * b + cl] : 0.0;
                x = mfma(ga, tb, x);
            }
#pragma unroll
            for (int s = 0; s < 4; s++) {  // Y = T_a X; X in D layout is the B operand of K-step s = v
                const int kk = 4 * s + g;
                const double ta = (cl <= kk) ? TG[(16 * a + cl) * LDT + 16 * a + kk] : 0.0;
                y = mfma(ta, x[s], y);
            }
#pragma unroll
            for (int v = 0; v < 4; v++) TG[(16 * a + g + 4 * v) * LDT + 16 * b + cl] = -y[v];
        }
        if constexpr (CT == 4) {
            // pairs of 32: rows {0,1} x columns {2,3}; wavefront w owns block (ia, jb)
            const int ia = (w >> 1) & 1, jb = 2 + (w & 1);
            const bool mw = w < 4;  // wavefronts 0..3 own the four blocks
            __syncthreads();
            d4 x = d4zero();
#pragma unroll
            for (int kb = 2; kb < 4; kb++) {
                if (kb > jb || !mw) continue;  // T_BB is upper triangular
#pragma unroll
                for (int s = 0; s < 4; s++) {
                    const int kk = 4 * s + g;
                    const double ga = TG[(16 * kb + kk) * LDT + 16 * ia + cl];
                    const double tb =
                        (kb < jb || kk <= cl) ? TG[(16 * kb + kk) * LDT + 16 * jb + cl] : 0.0;
                    x = mfma(ga, tb, x);
                }
            }
            if (mw) {
#pragma unroll
                for (int v = 0; v < 4; v++) TG[(16 * ia + g + 4 * v) * LDT + 16 * jb + cl] = x[v];
            }
            __syncthreads();
            d4 y = d4zero();
#pragma unroll
            for (int ka = 0; ka < 2; ka++) {
                if (ka < ia || !mw) continue;  // T_AA is upper triangular
#pragma unroll
                for (int s = 0; s < 4; s++) {
                    const int kk = 4 * s + g;
                    const double ta =
                        (ka > ia || cl <= kk) ? TG[(16 * ia + cl) * LDT + 16 * ka + kk] : 0.0;
                    y = mfma(ta, TG[(16 * ka + kk) * LDT + 16 * jb + cl], y);
                }
            }
            __syncthreads();  // every X block has been read
            if (mw) {
#pragma unroll
                for (int v = 0; v < 4; v++) TG[(16 * ia + g + 4 * v) * LDT + 16 * jb + cl] = -y[v];
            }
        }
    }
}

}  // namespace

// acc[rb][ct] += X[rows, :] B over the rows RPW w + 16 rb + (0..15) of a
// tile: X row-major (ld ldx), contraction index rows_kidx(s, g) (each batch
// of K-steps consumes whole 128-byte lines of the rows it touches; columns
// >= kmax read as zero), B a (4 KS) x (16 CT) matrix in B-operand order
// (k_permute_b).  K-steps are taken eight at a time, each B load
// serving every row block.
template <int RB, int CT, int KS>
__device__ __forceinline__ void rows_prod(d4 (&acc)[RB][CT], const double* __restrict__ X, int ldx, int row0,
                                          int trows, int kmax, const double* __restrict__ B, int l) {
    constexpr int SC = (KS < 8) ? KS : 8;
    const int g = l >> 4, cl = l & 15;
#pragma unroll 2
    for (int s0 = 0; s0 < KS; s0 += SC) {
        double a[RB][SC], b[SC][CT];
#pragma unroll
        for (int rb = 0; rb < RB; rb++) {
            const int xr = row0 + 16 * rb + cl;
#pragma unroll
            for (int s = 0; s < SC; s++) {
                const int kk = rows_kidx(s0 + s, g);
                a[rb][s] = (xr < trows && kk < kmax) ? X[xr * ldx + kk] : 0.0;
            }
        }
#pragma unroll
        for (int s = 0; s < SC; s++)
#pragma unroll
            for (int ct = 0; ct < CT; ct++) b[s][ct] = B[((s0 + s) * CT + ct) * 64 + l];
#pragma unroll
        for (int s = 0; s < SC; s++)
#pragma unroll
            for (int rb = 0; rb < RB; rb++)
#pragma unroll
                for (int ct = 0; ct < CT; ct++) acc[rb][ct] = mfma(a[rb][s], b[s][ct], acc[rb][ct]);
    }
}

// rows_prod for a full tile (every row present, kmax = 4 KS) with X 16-byte
// aligned and ldx even: no masks, so each lane reads its two adjacent
// columns of a K-step pair with one 16-byte load.
template <int RB, int CT, int KS>
__device__ __forceinline__ void rows_prod_full(d4 (&acc)[RB][CT], const double* __restrict__ X, int ldx, int row0,
                                               const double* __restrict__ B, int l) {
    constexpr int SC = 4;          // K-steps per batch: one 128-byte line of each row
    constexpr int NBT = KS / SC;   // batches
    static_assert(NBT * SC == KS, "KS must be a multiple of 4");
    const int g = l >> 4, cl = l & 15;
    // the loads of batch ib + 1 are issued before the MFMAs of batch ib
    auto load = [&](int s0, double(&a)[RB][SC], double(&b)[SC][CT]) {
#pragma unroll
        for (int rb = 0; rb < RB; rb++) {
            const double* xr = X + (row0 + 16 * rb + cl) * ldx;
#pragma unroll
            for (int s = 0; s < SC / 2; s++) {
                const double2 z = *(const double2*)(xr + rows_kidx(s0 + 2 * s, g));
                a[rb][2 * s] = z.x;
                a[rb][2 * s + 1] = z.y;
            }
        }
#pragma unroll
        for (int s = 0; s < SC; s++)
#pragma unroll
            for (int ct = 0; ct < CT; ct++) b[s][ct] = B[((s0 + s) * CT + ct) * 64 + l];
    };
    double a[2][RB][SC], b[2][SC][CT];
    load(0, a[0], b[0]);
#pragma unroll
    for (int ib = 0; ib < NBT; ib++) {
        const int cur = ib & 1;
        if (ib + 1 < NBT) load((ib + 1) * SC, a[cur ^ 1], b[cur ^ 1]);
#pragma unroll
        for (int s = 0; s < SC; s++)
#pragma unroll
            for (int rb = 0; rb < RB; rb++)
#pragma unroll
                for (int ct = 0; ct < CT; ct++) acc[rb][ct] = mfma(a[cur][rb][s], b[cur][s][ct], acc[rb][ct]);
    }
}

template <int KP, int K0P, int PANEL, int RBO, int NWT = NW>
__device__ __forceinline__ void leaf_chunk(const TsqrLevel& L, const int c) {
    constexpr int RB = Geo<KP, RBO, NWT>::RB, RPW = Geo<KP, RBO, NWT>::RPW, TB = Geo<KP, RBO, NWT>::TB;
    constexpr int CT = KP / 16;
    constexpr int LDT = KP + 1;
    constexpr bool HASV = K0P > 0;
    constexpr int KS0 = (K0P > 0) ? K0P / 4 : 1;
    constexpr int MT0 = (K0P > 0) ? K0P / 16 : 1;  // 16-column blocks of N^T
    constexpr int NJW = (MT0 + NWT - 1) / NWT;      // ... owned per wavefront

    extern __shared__ double sm[];
    double* TG = sm;                    // KP x LDT: T (upper) and Gm (strict lower)
    double* slot = TG + KP * LDT;       // KP x LDT: running R of the chunk
    double* xcol = slot + KP * LDT;     // TB: pivot column, RPW rows per wavefront
    double* prow = xcol + TB;           // 2 x KP: pivot row of the plain tile
    double* part = prow + 2 * KP;        // 2 x NWT x KP: partial dot products
    double* taus = part + 2 * NWT * KP;  // KP: tau of each reflector

    const int tid = threadIdx.x, w = tid >> 6;
    const int k = L.k;
    const int k0 = HASV ? L.k0 : 0;
    const int64_t cr0 = (int64_t)c * L.m / L.nchunk;
    const int64_t cr1 = (int64_t)(c + 1) * L.m / L.nchunk;
    const int ntiles = (int)((cr1 - cr0 + TB - 1) / TB);

    // The running N_c^T (KP x K0P, = Q_chunk^T V_chunk) lives in L.Nc[c];
    // wavefront w owns its 16-column blocks nj = w, w + NWT, ... (all rows) and
    // is the only one to read or write them.
    double* NT = (HASV && k0 > 0) ? L.Nc + (int64_t)c * KP * K0P : nullptr;

    // TG starts at zero, so that it only ever holds finite values (the T
    // sweep multiplies whole rows of it by zeros instead of masking)
    for (int e = tid; e < KP * LDT; e += blockDim.x) TG[e] = 0.0;

    for (int t = 0; t < ntiles; t++) {
        if (t > 0) __syncthreads();  // readers of TG from the last tile are done
        const int64_t r0 = cr0 + (int64_t)t * TB;
        const int trows = (int)((cr1 - r0 < TB) ? (cr1 - r0) : TB);
        const bool plain = (t == 0);
        PHASE_TS(t, 0);
        // uniform (scalar) bases of this tile; per-lane offsets stay 32-bit
        const double* __restrict__ Xt = L.X + r0 * L.ldx;
        double* __restrict__ Yt = L.Y + r0 * L.ldy;
        const double* __restrict__ Vt = HASV ? L.V + r0 * L.ldv : nullptr;
        const int ldx = (int)L.ldx, ldy = (int)L.ldy, ldv = (int)L.ldv;

        // ---- load the tile (rows r0.., in accumulator layout)
        d4 x[RB][CT];
        {
            const int l = opaque_lane(), cl = l & 15;
#pragma unroll
            for (int rb = 0; rb < RB; rb++)
#pragma unroll
                for (int ct = 0; ct < CT; ct++)
#pragma unroll
                    for (int v = 0; v < 4; v++) {
                        const int row = tile_row<RPW>(w, rb, l, v), col = 16 * ct + cl;
                        x[rb][ct][v] = (row < trows && col < k) ? Xt[row * ldx + col] : 0.0;
                    }
        }

        // ---- the update of A (Algorithm 1) on these rows: A <- A + V Z  (MFMA; Z is
        // read in B-operand order from L.Z, see k_permute_b)
        if (PANEL != PANEL_F64 && HASV && k0 > 0) {
            vprod_lowp<PANEL, RB, CT, (K0P > 0 ? K0P : 16)>(x, Vt, ldv, RPW * w, trows, k0, L.Zlp, opaque_lane());
        } else if (HASV && k0 > 0) {
            // a full tile with 16-byte aligned rows takes the unmasked, pipelined product
            const bool fullv = trows == TB && k0 == K0P && (ldv & 1) == 0 && (((uintptr_t)Vt) & 15) == 0;
            if constexpr (HASV) {
                if (fullv) rows_prod_full<RB, CT, KS0>(x, Vt, ldv, RPW * w, L.Z, opaque_lane());
            }
            const int l = opaque_lane(), g = l >> 4, cl = l & 15;
            constexpr int SC = 4;  // K-steps per chunk
#pragma unroll 2
            for (int s0 = 0; s0 < (fullv ? 0 : KS0); s0 += SC) {
                double a[RB][SC], b[SC][CT];
#pragma unroll
                for (int rb = 0; rb < RB; rb++) {
                    const int vr = RPW * w + 16 * rb + cl;  // A-operand row of this lane
#pragma unroll
                    for (int s = 0; s < SC; s++) {
                        const int kk = rows_kidx(s0 + s, g);  // a batch reads whole lines of V
                        a[rb][s] = (vr < trows && kk < k0) ? Vt[vr * ldv + kk] : 0.0;
                    }
                }
#pragma unroll
                for (int s = 0; s < SC; s++)
#pragma unroll
                    for (int ct = 0; ct < CT; ct++) b[s][ct] = L.Z[((s0 + s) * CT + ct) * 64 + l];
#pragma unroll
                for (int s = 0; s < SC; s++)
#pragma unroll
                    for (int rb = 0; rb < RB; rb++)
#pragma unroll
                        for (int ct = 0; ct < CT; ct++) x[rb][ct] = mfma(a[rb][s], b[s][ct], x[rb][ct]);
            }
        }

        PHASE_TS(t, 1);
        // ---- Householder QR of the tile (plain) or of [R; tile] (structured)
        double beta_last;
        if (plain) beta_last = householder_tile<KP, true, RBO, NWT>(x, k, w, xcol, prow, part, slot, TG, taus);
        else beta_last = householder_tile<KP, false, RBO, NWT>(x, k, w, xcol, prow, part, slot, TG, taus);
        __syncthreads();
        // row k-1 of the slot has no trailing columns; only its diagonal changes
        if (!plain && w == 0 && k > 0 && (threadIdx.x & 63) == k - 1) slot[(k - 1) * LDT + (k - 1)] = beta_last;
        PHASE_TS(t, 2);
        // tile outputs first (R -> slot, registers -> Y), so that the tile
        // registers are free during the T factor
        {
            const int l = opaque_lane(), cl = l & 15;
            if (plain) {
                // R -> slot; registers -> unit lower trapezoidal Y
#pragma unroll
                for (int rb = 0; rb < RB; rb++)
#pragma unroll
                    for (int ct = 0; ct < CT; ct++)
#pragma unroll
                        for (int v = 0; v < 4; v++) {
                            const int row = tile_row<RPW>(w, rb, l, v), col = 16 * ct + cl;
                            if (row < KP && col < KP) {
                                const double xv = x[rb][ct][v];
                                slot[row * LDT + col] = (col >= row && row < k && col < k) ? xv : 0.0;
                                if (col > row) x[rb][ct][v] = 0.0;
                                else if (col == row) x[rb][ct][v] = (row < k) ? 1.0 : 0.0;
                            }
                        }
            }
#pragma unroll
            for (int rb = 0; rb < RB; rb++)
#pragma unroll
                for (int ct = 0; ct < CT; ct++)
#pragma unroll
                    for (int v = 0; v < 4; v++) {
                        const int row = tile_row<RPW>(w, rb, l, v), col = 16 * ct + cl;
                        if (row < trows && col < k) Yt[row * ldy + col] = x[rb][ct][v];
                    }
        }
        PHASE_TS(t, 5);
        // compact-WY factor (H_0 ... H_{k-1} = I - U T U^T):
        //   T(i,i) = tau_i,  T(i,j) = -tau_j sum_{i<=p<j} T(i,p) u_p^T u_j
        // in 16 x 16 blocks.  Each diagonal block is the factor of its own 16
        // reflectors (the recurrence above, wavefront b for block b); two
        // adjacent factors merge as
        //   [T_a  X; 0  T_b],  X = -T_a (U_a^T U_b) T_b,
        // first in pairs of 16 columns, then in pairs of 32, on MFMA.  The
        // Gram U^T U sits in the strict lower triangle of TG (G(p, j) at
        // TG[j][p]); T goes to the upper triangle.
        tile_t_factor<KP>(TG, taus, k, w);
        PHASE_TS(t, 4);
        __syncthreads();  // T complete, Y rows visible to the whole workgroup
        PHASE_TS(t, 6);
        {
            const int64_t ti = (int64_t)c * L.maxtiles + t;
            double* Tg = L.Tt + ti * KP * KP;
            for (int e = tid; e < KP * KP; e += blockDim.x) {
                const int i = e / KP, jj = e % KP;
                Tg[e] = (jj >= i && jj < k) ? TG[i * LDT + jj] : 0.0;
            }
        }
        PHASE_TS(t, 3);

        // ---- level 0: N_c^T <- Q^T V of the chunk so far, through
        //   structured tile:  N^T <- N^T - T^T (N^T + Y^T V)
        //   plain tile 0:     N^T  = V_0[0:k] - L_0 T^T (Y^T V),  L_0 = Y_0[0:k, 0:k]
        if (HASV && k0 > 0) {
            const int l = opaque_lane(), g = l >> 4, cl = l & 15;
            // S^T = N^T + Y^T V (structured) or Y^T V (plain); the N^T loads are
            // issued first so that they overlap the product loop
            d4 sacc[CT][NJW];
#pragma unroll
            for (int mi = 0; mi < CT; mi++)
#pragma unroll
                for (int q = 0; q < NJW; q++)
#pragma unroll
                    for (int v = 0; v < 4; v++) {
                        const int r = 16 * mi + drow(l, v), cc = 16 * (w + NWT * q) + cl;
                        sacc[mi][q][v] = (!plain && cc < K0P) ? NT[r * K0P + cc] : 0.0;
                    }
            // B^T = Y^T V over the tile rows (4 rows per K-step)
            constexpr int US = 4;  // K-steps per batch of loads (the tile registers are free here)
            for (int s0 = 0; s0 < TB / 4; s0 += US) {
                double ya[US][CT], vb[US][NJW];
#pragma unroll
                for (int u = 0; u < US; u++) {
                    const int row = 4 * (s0 + u) + g;
                    const bool ok = row < trows;
#pragma unroll
                    for (int mi = 0; mi < CT; mi++) {
                        const int yc = 16 * mi + cl;
                        ya[u][mi] = (ok && yc < k) ? Yt[row * ldy + yc] : 0.0;
                    }
#pragma unroll
                    for (int q = 0; q < NJW; q++) {
                        const int vc = 16 * (w + NWT * q) + cl;
                        vb[u][q] = (ok && vc < k0) ? Vt[row * ldv + vc] : 0.0;
                    }
                }
#pragma unroll
                for (int u = 0; u < US; u++)
#pragma unroll
                    for (int mi = 0; mi < CT; mi++)
#pragma unroll
                        for (int q = 0; q < NJW; q++) sacc[mi][q] = mfma(ya[u][mi], vb[u][q], sacc[mi][q]);
            }
            // D^T = T^T S^T, contracting over the rows of S^T (K-step (rb, v)
            // takes rows 16 rb + l/16 + 4 v, i.e. register v of block rb)
            d4 dacc[CT][NJW];
#pragma unroll
            for (int mi = 0; mi < CT; mi++)
#pragma unroll
                for (int q = 0; q < NJW; q++) dacc[mi][q] = d4zero();
#pragma unroll
            for (int rb = 0; rb < CT; rb++)
#pragma unroll
                for (int v = 0; v < 4; v++) {
                    const int p = 16 * rb + drow(l, v);
#pragma unroll
                    for (int mi = 0; mi < CT; mi++) {
                        if (rb > mi) continue;  // T^T is lower triangular
                        const int m = 16 * mi + cl;
                        const double a = (p <= m && m < k) ? TG[p * LDT + m] : 0.0;  // T^T(m, p)
#pragma unroll
                        for (int q = 0; q < NJW; q++) dacc[mi][q] = mfma(a, sacc[rb][q][v], dacc[mi][q]);
                    }
                }
            if (!plain) {
#pragma unroll
                for (int mi = 0; mi < CT; mi++)
#pragma unroll
                    for (int q = 0; q < NJW; q++)
#pragma unroll
                        for (int v = 0; v < 4; v++) {
                            const int r = 16 * mi + drow(l, v), cc = 16 * (w + NWT * q) + cl;
                            if (cc < K0P) NT[r * K0P + cc] -= dacc[mi][q][v];
                        }
            } else {
                // E^T = L_0 D^T, N^T = V_0[0:k] - E^T
                d4 eacc[CT][NJW];
#pragma unroll
                for (int mi = 0; mi < CT; mi++)
#pragma unroll
                    for (int q = 0; q < NJW; q++) eacc[mi][q] = d4zero();
#pragma unroll
                for (int rb = 0; rb < CT; rb++)
#pragma unroll
                    for (int v = 0; v < 4; v++) {
                        const int p = 16 * rb + drow(l, v);
#pragma unroll
                        for (int mi = 0; mi < CT; mi++) {
                            if (rb > mi) continue;  // L_0 is lower triangular
                            const int m = 16 * mi + cl;
                            const double a = (m < k && p < k) ? Yt[m * ldy + p] : 0.0;  // L_0(m, p)
#pragma unroll
                            for (int q = 0; q < NJW; q++) eacc[mi][q] = mfma(a, dacc[rb][q][v], eacc[mi][q]);
                        }
                    }
#pragma unroll
                for (int mi = 0; mi < CT; mi++)
#pragma unroll
                    for (int q = 0; q < NJW; q++)
#pragma unroll
                        for (int v = 0; v < 4; v++) {
                            const int r = 16 * mi + drow(l, v), cc = 16 * (w + NWT * q) + cl;
                            const double vt = (r < k && cc < k0) ? Vt[r * ldv + cc] : 0.0;
                            if (cc < K0P) NT[r * K0P + cc] = vt - eacc[mi][q][v];
                        }
            }
        }
    }
    PHASE_TS(63, 0);

    // ---- chunk output: R_c into the next level
    for (int e = tid; e < k * KP; e += blockDim.x) {
        const int i = e / KP, jj = e % KP;
        L.Rnext[((int64_t)c * k + i) * L.ldrn + jj] = (jj < k && jj >= i) ? slot[i * LDT + jj] : 0.0;
    }
}


// Form the explicit Q of one level from the stored Householder vectors:
// chunk c's rows of Q are Q_chunk G_c, with G_c read from the formed level
// above (or the phase signs at the top).  Tiles are visited last to first;
// C carries G_c down the flat tree:
//   structured tile t:  K = T_t C,                rows = -Y_t K,  C <- C - K
//   plain tile 0:       K = T_0 (Y_0[0:k]^T C),   rows = [C; 0] - Y_0 K
// Level 0 adds V N (formation of Q in Algorithm 1: Q_low = Q_ + V_low N).
// Output rows overwrite the Householder vectors in place.
template <int KP, int K0P, int PANEL, int RBO, int NWT = NW>
__device__ __forceinline__ void form_chunk(const TsqrLevel& L, const int c) {
    constexpr int RB = Geo<KP, RBO, NWT>::RB, RPW = Geo<KP, RBO, NWT>::RPW, TB = Geo<KP, RBO, NWT>::TB;
    constexpr int CT = KP / 16;
    constexpr int LDT = KP + 1;
    constexpr bool HASV = K0P > 0;
    constexpr int KS0 = (K0P > 0) ? K0P / 4 : 1;
    constexpr int KSK = KP / 4;
    constexpr int NTK = CT * CT;
    constexpr int NTKW = (NTK + NWT - 1) / NWT;

    extern __shared__ double sm[];
    double* Cm = sm;              // KP x LDT
    double* Kp = Cm + KP * LDT;   // KP x LDT region: E (plain) then -K permuted
    const double* Np = L.Nglob;   // N in B-operand order (see k_permute_b)

    const int tid = threadIdx.x, w = tid >> 6;
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
    }
    __syncthreads();

    for (int t = ntiles - 1; t >= 0; t--) {
        const int64_t r0 = cr0 + (int64_t)t * TB;
        const int trows = (int)((cr1 - r0 < TB) ? (cr1 - r0) : TB);
        const bool plain = (t == 0);
        const double* Tg = L.Tt + ((int64_t)c * L.maxtiles + t) * KP * KP;
        double* __restrict__ Yt = L.Y + r0 * L.ldy;
        const double* __restrict__ Vt = HASV ? L.V + r0 * L.ldv : nullptr;
        const int ldy = (int)L.ldy, ldv = (int)L.ldv;
        const int l = opaque_lane(), g = l >> 4, cl = l & 15;

        const double* src = Cm;
        if (plain) {
            d4 e[NTKW];
#pragma unroll
            for (int i = 0; i < NTKW; i++) e[i] = d4zero();
#pragma unroll
            for (int s = 0; s < KSK; s++)
#pragma unroll
                for (int i = 0; i < NTKW; i++) {
                    const int id = w + NWT * i;
                    if (id < NTK) {
                        const int mi = id / CT, nj = id % CT;
                        const int yr = 4 * s + g, yc = 16 * mi + cl;
                        const double a = (yr < k && yc < k) ? Yt[yr * ldy + yc] : 0.0;
                        e[i] = mfma(a, Cm[(4 * s + g) * LDT + 16 * nj + cl], e[i]);
                    }
                }
#pragma unroll
            for (int i = 0; i < NTKW; i++) {
                const int id = w + NWT * i;
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
        // contraction index split as g * KSK + s: a lane reads KSK consecutive
        // entries of one row of T_t (one 128-byte piece per lane group)
#pragma unroll
        for (int s = 0; s < KSK; s++)
#pragma unroll
            for (int i = 0; i < NTKW; i++) {
                const int id = w + NWT * i;
                if (id < NTK) {
                    const int mi = id / CT, nj = id % CT;
                    const double a = Tg[(16 * mi + cl) * KP + g * KSK + s];
                    kk[i] = mfma(a, src[(g * KSK + s) * LDT + 16 * nj + cl], kk[i]);
                }
            }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NTKW; i++) {
            const int id = w + NWT * i;
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
                    const int row = tile_row<RPW>(w, rb, l, v), col = 16 * ct + cl;
                    acc[rb][ct][v] = (plain && row < k && col < k) ? Cm[row * LDT + col] : 0.0;
                }
#pragma unroll
        for (int rb = 0; rb < RB; rb++) {
            const int yr = RPW * w + 16 * rb + cl;
            const bool ok = yr < trows;
            {
                const double* yp = Yt + yr * ldy + g * KSK;
                double a[KSK];
#pragma unroll
                for (int s = 0; s < KSK; s++) a[s] = (ok && g * KSK + s < k) ? yp[s] : 0.0;
#pragma unroll
                for (int s = 0; s < KSK; s++)
#pragma unroll
                    for (int ct = 0; ct < CT; ct++)
                        acc[rb][ct] = mfma(a[s], Kp[(s * CT + ct) * 64 + l], acc[rb][ct]);
            }
        }
        // + V N: K-steps outer so that each B-operand load of N serves every
        // row block (N is read in operand order, see k_permute_b)
        if (PANEL == PANEL_F64 && HASV && k0 > 0) {
            constexpr int SC = 4;  // K-steps per batch of loads
#pragma unroll 2
            for (int s0 = 0; s0 < KS0; s0 += SC) {
                double a[RB][SC], b[SC][CT];
#pragma unroll
                for (int rb = 0; rb < RB; rb++) {
                    const int yr = RPW * w + 16 * rb + cl;
#pragma unroll
                    for (int s = 0; s < SC; s++) {
                        const int kk = rows_kidx(s0 + s, g);
                        a[rb][s] = (yr < trows && kk < k0) ? Vt[yr * ldv + kk] : 0.0;
                    }
                }
#pragma unroll
                for (int s = 0; s < SC; s++)
#pragma unroll
                    for (int ct = 0; ct < CT; ct++) b[s][ct] = Np[((s0 + s) * CT + ct) * 64 + l];
#pragma unroll
                for (int s = 0; s < SC; s++)
#pragma unroll
                    for (int rb = 0; rb < RB; rb++)
#pragma unroll
                        for (int ct = 0; ct < CT; ct++) acc[rb][ct] = mfma(a[rb][s], b[s][ct], acc[rb][ct]);
            }
        }
        if (PANEL != PANEL_F64 && HASV && k0 > 0)
            vprod_lowp<PANEL, RB, CT, (K0P > 0 ? K0P : 16)>(acc, Vt, ldv, RPW * w, trows, k0, L.Nlp, l);
#pragma unroll
        for (int rb = 0; rb < RB; rb++)
#pragma unroll
            for (int ct = 0; ct < CT; ct++)
#pragma unroll
                for (int v = 0; v < 4; v++) {
                    const int row = tile_row<RPW>(w, rb, l, v), col = 16 * ct + cl;
                    if (row < trows && col < k) Yt[row * ldy + col] = acc[rb][ct][v];
                }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Formation of level 0 in two passes.  The only sequential dependence of the
// flat-tree formation is through the k x k block C that each tile hands to the
// one above it (top-down: K_t = T_t C, C <- C - K_t for a structured tile;
// K_0 = T_0 L_0^T C for the plain tile 0, whose top k rows also receive C).
// kchain_chunk walks that recurrence for one chunk and overwrites every T_t
// in place with -K_t (in B-operand order, K split by rows_kidx) and stores the
// final C; rows_tile then forms the Q rows of any tile on its own,
//   Q_t = [C; 0] (tile 0 only) - Y_t K_t + V_t N,
// with no barrier and no shared memory, so that the streaming MFMA work runs
// at full occupancy over every tile of every chunk at once.

template <int KP>
struct KchainLds {
    static constexpr int LDT = KP + 1;
    static constexpr int total = 2 * KP * LDT;
};

template <int KP>
__device__ __forceinline__ void kchain_chunk(const TsqrLevel& L, const int c) {
    constexpr int TB = Geo<KP>::TB;
    constexpr int CT = KP / 16;
    constexpr int LDT = KP + 1;
    constexpr int KSK = KP / 4;
    constexpr int NTK = CT * CT;
    constexpr int NTKW = (NTK + NW - 1) / NW;
    constexpr int PT = KP * KP / (NW * 64);  // entries of T_t per thread
    static_assert(PT * NW * 64 == KP * KP, "one T_t per workgroup pass");

    extern __shared__ double sm[];
    double* Cm = sm;             // KP x LDT: the running C
    double* Tb = Cm + KP * LDT;  // KP x LDT: T_t (structured tiles), L_0^T C (plain tile)

    const int tid = threadIdx.x, w = tid >> 6;
    const int k = L.k;
    const int64_t cr0 = (int64_t)c * L.m / L.nchunk;
    const int64_t cr1 = (int64_t)(c + 1) * L.m / L.nchunk;
    const int ntiles = (int)((cr1 - cr0 + TB - 1) / TB);
    {
        const double* G = L.Gin + (int64_t)c * L.gstride * L.ldg;
        for (int e = tid; e < KP * KP; e += blockDim.x) {
            const int i = e / KP, jj = e % KP;
            Cm[i * LDT + jj] = (i < k && jj < k) ? G[(int64_t)i * L.ldg + jj] : 0.0;
        }
    }
    // T_t of the next structured tile is fetched one step ahead (PT values
    // per thread) and staged into Tb once the current step has read it
    double tp[PT];
    auto fetch = [&](int t) {
        const double* Tg = L.Tt + ((int64_t)c * L.maxtiles + t) * KP * KP;
#pragma unroll
        for (int q = 0; q < PT; q++) tp[q] = Tg[tid + q * NW * 64];
    };
    auto stage = [&]() {
#pragma unroll
        for (int q = 0; q < PT; q++) {
            const int e = tid + q * NW * 64;
            Tb[(e / KP) * LDT + e % KP] = tp[q];
        }
    };
    if (ntiles > 1) {
        fetch(ntiles - 1);
        stage();
    }
    __syncthreads();
    const int l = lane_id(), g = l >> 4, cl = l & 15;

    for (int t = ntiles - 1; t >= 0; t--) {
        const bool plain = (t == 0);
        double* Kg = L.Tt + ((int64_t)c * L.maxtiles + t) * KP * KP;
        d4 kk[NTKW];
#pragma unroll
        for (int i = 0; i < NTKW; i++) kk[i] = d4zero();
        if (!plain) {
            if (t > 1) fetch(t - 1);
            // K = T_t C, contraction index 4 s + g; T_t is upper triangular, so
            // row block mi starts at K-step 4 mi
#pragma unroll
            for (int i = 0; i < NTKW; i++) {
                const int id = w + NW * i;
                if (id < NTK) {
                    const int mi = id / CT, nj = id % CT;
#pragma unroll 4
                    for (int s = 4 * mi; s < KSK; s++)
                        kk[i] = mfma(Tb[(16 * mi + cl) * LDT + 4 * s + g], Cm[(4 * s + g) * LDT + 16 * nj + cl], kk[i]);
                }
            }
        } else {
            // E = L_0^T C with L_0 = Y_0[0:k, 0:k] (unit lower triangular) into Tb
            const double* Y0 = L.Y + cr0 * L.ldy;
            const int ldy = (int)L.ldy;
            d4 e[NTKW];
#pragma unroll
            for (int i = 0; i < NTKW; i++) e[i] = d4zero();
#pragma unroll 4
            for (int s = 0; s < KSK; s++)
#pragma unroll
                for (int i = 0; i < NTKW; i++) {
                    const int id = w + NW * i;
                    if (id < NTK) {
                        const int mi = id / CT, nj = id % CT;
                        const int yr = 4 * s + g, yc = 16 * mi + cl;
                        const double a = (yr < k && yc < k) ? Y0[yr * ldy + yc] : 0.0;
                        e[i] = mfma(a, Cm[(4 * s + g) * LDT + 16 * nj + cl], e[i]);
                    }
                }
#pragma unroll
            for (int i = 0; i < NTKW; i++) {
                const int id = w + NW * i;
                if (id < NTK) {
                    const int mi = id / CT, nj = id % CT;
#pragma unroll
                    for (int v = 0; v < 4; v++) Tb[(16 * mi + drow(l, v)) * LDT + 16 * nj + cl] = e[i][v];
                }
            }
            __syncthreads();
            // K = T_0 E (T_0 straight from its slot)
#pragma unroll 4
            for (int s = 0; s < KSK; s++)
#pragma unroll
                for (int i = 0; i < NTKW; i++) {
                    const int id = w + NW * i;
                    if (id < NTK) {
                        const int mi = id / CT, nj = id % CT;
                        kk[i] = mfma(Kg[(16 * mi + cl) * KP + g * KSK + s], Tb[(g * KSK + s) * LDT + 16 * nj + cl],
                                     kk[i]);
                    }
                }
        }
        __syncthreads();  // every read of C, Tb and T_t is done
#pragma unroll
        for (int i = 0; i < NTKW; i++) {
            const int id = w + NW * i;
            if (id < NTK) {
                const int mi = id / CT, nj = id % CT;
#pragma unroll
                for (int v = 0; v < 4; v++) {
                    const int r = 16 * mi + drow(l, v), cc = 16 * nj + cl;
                    // row r of K is K-step s, lane group g with r = rows_kidx(s, g)
                    Kg[((2 * (r >> 3) + (r & 1)) * CT + nj) * 64 + 16 * ((r >> 1) & 3) + cl] = -kk[i][v];
                    if (!plain) Cm[r * LDT + cc] -= kk[i][v];
                }
            }
        }
        if (!plain && t > 1) stage();
        __syncthreads();
    }
    // C as the plain tile 0 sees it (zero outside the k x k block)
    double* Cf = L.Cfin + (int64_t)c * KP * KP;
    for (int e = tid; e < KP * KP; e += blockDim.x) Cf[e] = Cm[(e / KP) * LDT + e % KP];
}

template <int KP, int K0P, int PANEL>
__device__ __forceinline__ void rows_tile(const TsqrLevel& L, const int c, const int t) {
    constexpr int RB = Geo<KP>::RB, RPW = Geo<KP>::RPW, TB = Geo<KP>::TB;
    constexpr int CT = KP / 16;
    constexpr int KSK = KP / 4;
    constexpr bool HASV = K0P > 0;
    constexpr int KS0 = (K0P > 0) ? K0P / 4 : 1;

    const int w = threadIdx.x >> 6;
    const int k = L.k;
    const int k0 = HASV ? L.k0 : 0;
    const int64_t cr0 = (int64_t)c * L.m / L.nchunk;
    const int64_t cr1 = (int64_t)(c + 1) * L.m / L.nchunk;
    const int64_t r0 = cr0 + (int64_t)t * TB;
    if (r0 >= cr1) return;  // slot beyond this chunk's tiles (uniform)
    const int trows = (int)((cr1 - r0 < TB) ? (cr1 - r0) : TB);
    const double* __restrict__ Kg = L.Tt + ((int64_t)c * L.maxtiles + t) * KP * KP;  // -K_t
    double* __restrict__ Yt = L.Y + r0 * L.ldy;
    const double* __restrict__ Vt = HASV ? L.V + r0 * L.ldv : nullptr;
    const int ldy = (int)L.ldy, ldv = (int)L.ldv;
    const int l = lane_id(), g = l >> 4, cl = l & 15;

    d4 acc[RB][CT];
    if (t == 0) {
        const double* Cf = L.Cfin + (int64_t)c * KP * KP;
#pragma unroll
        for (int rb = 0; rb < RB; rb++)
#pragma unroll
            for (int ct = 0; ct < CT; ct++)
#pragma unroll
                for (int v = 0; v < 4; v++) {
                    const int row = tile_row<RPW>(w, rb, l, v), col = 16 * ct + cl;
                    acc[rb][ct][v] = (row < KP) ? Cf[row * KP + col] : 0.0;
                }
    } else {
#pragma unroll
        for (int rb = 0; rb < RB; rb++)
#pragma unroll
            for (int ct = 0; ct < CT; ct++) acc[rb][ct] = d4zero();
    }
    // a full tile with 16-byte aligned rows takes the unmasked paths
    const bool full = trows == TB && k == KP && (!HASV || k0 == K0P) && ((ldy | (HASV ? ldv : 0)) & 1) == 0 &&
                      ((((uintptr_t)Yt) | ((uintptr_t)Vt)) & 15) == 0;
    // - Y_t K_t (-K_t in B-operand order from the K chain)
    if (full) rows_prod_full<RB, CT, KSK>(acc, Yt, ldy, RPW * w, Kg, l);
    else rows_prod<RB, CT, KSK>(acc, Yt, ldy, RPW * w, trows, k, Kg, l);
    // + V_t N (N in B-operand order, see k_permute_b)
    if constexpr (PANEL == PANEL_F64 && HASV) {
        if (k0 > 0) {
            if (full) rows_prod_full<RB, CT, KS0>(acc, Vt, ldv, RPW * w, L.Nglob, l);
            else rows_prod<RB, CT, KS0>(acc, Vt, ldv, RPW * w, trows, k0, L.Nglob, l);
        }
    }
    if (PANEL != PANEL_F64 && HASV && k0 > 0)
        vprod_lowp<PANEL, RB, CT, (K0P > 0 ? K0P : 16)>(acc, Vt, ldv, RPW * w, trows, k0, L.Nlp, l);
    // each wavefront reads and writes only its own rows: no barrier
#pragma unroll
    for (int rb = 0; rb < RB; rb++)
#pragma unroll
        for (int ct = 0; ct < CT; ct++)
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int row = tile_row<RPW>(w, rb, l, v), col = 16 * ct + cl;
                if (row < trows && col < k) Yt[row * ldy + col] = acc[rb][ct][v];
            }
}

}  // namespace tho
