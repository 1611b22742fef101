// Level 0 of the complex chunked Householder QR with the generalized
// Householder step of Algorithm 1 fused in (complex128, gfx950).
//
// The same structure as the real leaf (tsqr_dev.h) in complex arithmetic:
// one workgroup of four wavefronts per row chunk walks the chunk in tiles of
// ZGeo::TB rows, the tile held in registers in the FP64 MFMA accumulator
// layout as separate real and imaginary parts.  Per tile:
//   A' = A_low + V_low Z on MFMA (four real products per complex one);
//   Householder QR of the tile (tile 0) or of [R; tile] with one workgroup
//   barrier per column; the reflectors follow the complex LAPACK convention
//   H = I - tau u u^H, beta = -sign(Re alpha) ||x|| real, u_j = 1;
//   T factor of the tile (H_0 ... H_{k-1} = I - U T U^H) by the column
//   recurrence from the Gram of the vectors;
//   the chain M <- M - T^H (M + Y^H V) (plain tile: M = V_0[0:k] - L_0 T^H
//   Y^H V), so that M_c = Q_chunk^H V_chunk and V_low^H Q_ = sum_c M_c^H G_c
//   need no further pass over V.
// The outputs (vectors in Y with an explicit unit diagonal in tile 0, T_t
// row-major, the chunk R) have the layout of the LDS leaf in k_complex.hip,
// whose formation kernels and upper levels take them unchanged.
#include "tho_device.h"
#include "tho_internal.h"

namespace tho {

namespace {

constexpr int ZNW = 4;  // wavefronts per workgroup

template <int KP>
struct ZGeo {
    static constexpr int CT = KP / 16;               // 16-column blocks
    static constexpr int RB = (KP >= 32) ? 2 : 4;    // 16-row blocks per wavefront
    static constexpr int RPW = 16 * RB;              // rows per wavefront
    static constexpr int TB = ZNW * RPW;             // rows per tile
    static constexpr int LDT = KP + 1;
};

template <int KP>
struct ZLeafLds {
    static constexpr int LDT = KP + 1;
    // slot (re, im), Gram (re, im), T (re, im), pivot column (re, im), pivot
    // row (re, im, two buffers), partial sums (re, im, two buffers), tau (re, im)
    static constexpr int total = 6 * KP * LDT + 2 * ZGeo<KP>::TB + 4 * KP + 4 * ZNW * KP + 2 * KP;
};

__device__ __forceinline__ int zlane() {
    int x = threadIdx.x & 63;
    asm volatile("" : "+v"(x));
    return x;
}

template <int RPW>
__device__ __forceinline__ int ztile_row(int w, int rb, int l, int v) {
    return RPW * w + 16 * rb + drow(l, v);
}

__device__ __forceinline__ double2 ld2(const double* p) { return *(const double2*)p; }
__device__ __forceinline__ void st2(double* p, double a, double b) { *(double2*)p = make_double2(a, b); }

struct ZShm {
    double *sr, *si;    // running R (slot)
    double *gr, *gi;    // Gram: G(p, j) = u_p^H u_j at [j][p] (p < j)
    double *tlr, *tli;  // T of the tile, T(p, m) at [p][m]
    double *xr, *xi;    // pivot column, RPW rows per wavefront
    double *prr, *pri;  // pivot row (plain tile), two buffers
    double *ptr, *pti;  // partial dot products, two buffers
    double *tar, *tai;  // tau
};

struct ZCarry {
    double beta_prev;
    double rnr, rni;  // structured: my entry of the previous pivot row after its reflector
    double msr, msi;  // scale 1 / (alpha - beta) of the reflector of column `lane` (0 until then)
};

// Columns 16 CTJ .. of the complex Householder QR of the register tile
// (PLAIN: the tile alone; otherwise [slot; tile]).  Per column j every
// wavefront forms, over its sub rows, d_c = sum conj(x_j) x_c for every
// column c; with the pivot-row values p_c, u = [1; x_sub s] (s = 1 / (alpha
// - beta)) gives sigma^2 = Re d_j and w_c = u^H x_c = p_c + conj(s) d_c.
// H^H is applied: x_c -= conj(tau) w_c u.  The vectors stay unscaled in the
// registers (scaled once after the loop); for c < j, s_c w_c = u_j^H u_c.
template <int KP, bool PLAIN, int CTJ>
__device__ __forceinline__ void zhh_block(d4 (&xr)[ZGeo<KP>::RB][KP / 16], d4 (&xi)[ZGeo<KP>::RB][KP / 16], int k,
                                          int w, const ZShm& S, ZCarry& cy) {
    constexpr int RB = ZGeo<KP>::RB, RPW = ZGeo<KP>::RPW, CT = KP / 16, LDT = KP + 1;
    const int l = zlane(), g = l >> 4, cl = l & 15;
    double* xwr = S.xr + RPW * w;
    double* xwi = S.xi + RPW * w;
    const int jend = (16 * CTJ + 16 < k) ? 16 * CTJ + 16 : k;
    for (int j = 16 * CTJ; j < jend; j++) {
        const int pb = j & 1, clj = j & 15;
        if (cl == clj) {
#pragma unroll
            for (int rb = 0; rb < RB; rb++)
#pragma unroll
                for (int v = 0; v < 4; v++) {
                    xwr[rb * 16 + g * 4 + v] = xr[rb][CTJ][v];
                    xwi[rb * 16 + g * 4 + v] = xi[rb][CTJ][v];
                }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        double sr_[RB][4], si_[RB][4];  // pivot column on my sub rows, 0 elsewhere
#pragma unroll
        for (int rb = 0; rb < RB; rb++)
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const bool sub = !PLAIN || ztile_row<RPW>(w, rb, l, v) > j;
                sr_[rb][v] = sub ? xwr[rb * 16 + g * 4 + v] : 0.0;
                si_[rb][v] = sub ? xwi[rb * 16 + g * 4 + v] : 0.0;
            }
        {
            double dr[CT], di[CT];
#pragma unroll
            for (int ct = 0; ct < CT; ct++) dr[ct] = di[ct] = 0.0;
#pragma unroll
            for (int rb = 0; rb < RB; rb++)
#pragma unroll
                for (int v = 0; v < 4; v++)
#pragma unroll
                    for (int ct = 0; ct < CT; ct++) {
                        // conj(s) x = (sr xr + si xi) + i (sr xi - si xr)
                        dr[ct] += sr_[rb][v] * xr[rb][ct][v];
                        dr[ct] += si_[rb][v] * xi[rb][ct][v];
                        di[ct] += sr_[rb][v] * xi[rb][ct][v];
                        di[ct] -= si_[rb][v] * xr[rb][ct][v];
                    }
            const double tr = col_sums<CT>(dr), ti = col_sums<CT>(di);  // valid in lanes l < KP
            if (l < KP) {
                S.ptr[(pb * ZNW + w) * KP + l] = tr;
                S.pti[(pb * ZNW + w) * KP + l] = ti;
            }
        }
        if (PLAIN && w == j / RPW) {
#pragma unroll
            for (int rb = 0; rb < RB; rb++)
#pragma unroll
                for (int v = 0; v < 4; v++)
                    if (ztile_row<RPW>(w, rb, l, v) == j) {
#pragma unroll
                        for (int ct = 0; ct < CT; ct++) {
                            S.prr[pb * KP + 16 * ct + cl] = xr[rb][ct][v];
                            S.pri[pb * KP + 16 * ct + cl] = xi[rb][ct][v];
                        }
                    }
        }
        __syncthreads();

        if (!PLAIN && j > 0 && w == 0) {
            if (l > j - 1 && l < k) {
                S.sr[(j - 1) * LDT + l] = cy.rnr;
                S.si[(j - 1) * LDT + l] = cy.rni;
            }
            if (l == j - 1) {
                S.sr[(j - 1) * LDT + (j - 1)] = cy.beta_prev;
                S.si[(j - 1) * LDT + (j - 1)] = 0.0;
            }
        }
        double dlr = 0.0, dli = 0.0, plr = 0.0, pli = 0.0;
        if (l < KP) {
            double qr[ZNW], qi[ZNW];
#pragma unroll
            for (int ww = 0; ww < ZNW; ww++) {
                qr[ww] = S.ptr[(pb * ZNW + ww) * KP + l];
                qi[ww] = S.pti[(pb * ZNW + ww) * KP + l];
            }
            plr = PLAIN ? S.prr[pb * KP + l] : S.sr[j * LDT + l];
            pli = PLAIN ? S.pri[pb * KP + l] : S.si[j * LDT + l];
#pragma unroll
            for (int ww = 0; ww < ZNW; ww++) {
                dlr += qr[ww];
                dli += qi[ww];
            }
        }
        const double sig2 = bcast(dlr, j);
        const double ar = bcast(plr, j), ai = bcast(pli, j);
        double beta = ar, tr = 0.0, ti = 0.0, scr = 0.0, sci = 0.0;
        if (sig2 != 0.0 || ai != 0.0) {
            const double nrm = sqrt(fma(ar, ar, fma(ai, ai, sig2)));
            beta = (ar < 0.0) ? nrm : -nrm;
            const double rb_ = 1.0 / beta;
            tr = (beta - ar) * rb_;  // tau = (beta - alpha) / beta
            ti = -ai * rb_;
            // s = 1 / (alpha - beta) = conj(alpha - beta) / |alpha - beta|^2
            const double er = ar - beta;
            const double den = 1.0 / fma(er, er, ai * ai);
            scr = er * den;
            sci = -ai * den;
        }
        // w_c = p_c + conj(s) d_c
        const double wr = plr + (scr * dlr + sci * dli);
        const double wi = pli + (scr * dli - sci * dlr);
        // conj(tau) w
        const double cwr = tr * wr + ti * wi, cwi = tr * wi - ti * wr;
        if (!PLAIN) {
            cy.rnr = plr - cwr;
            cy.rni = pli - cwi;
        }
        if (w == 0) {
            if (l < j) {
                // G(l, j) = u_l^H u_j = conj(s_l w_l)
                S.gr[j * LDT + l] = cy.msr * wr - cy.msi * wi;
                S.gi[j * LDT + l] = -(cy.msr * wi + cy.msi * wr);
            }
            if (l == 0) {
                S.tar[j] = tr;
                S.tai[j] = ti;
            }
        }
        if (l == j) {
            cy.msr = scr;
            cy.msi = sci;
        }
        double gvr[4], gvi[4];
        gather_cols(cwr, gvr);
        gather_cols(cwi, gvi);
        // x_c -= u (conj(tau) w_c): plain u = 1 on the pivot row, s x_sub
        // below; structured u = s x_sub, so the coefficient takes s
#pragma unroll
        for (int ct = CTJ; ct < CT; ct++) {
            double kr = gvr[ct], ki = gvi[ct];
            if (!PLAIN) {
                const double t0 = scr * kr - sci * ki;
                ki = scr * ki + sci * kr;
                kr = t0;
            }
            if (!(ct > CTJ || cl > clj)) {
                kr = 0.0;
                ki = 0.0;
            }
#pragma unroll
            for (int rb = 0; rb < RB; rb++)
#pragma unroll
                for (int v = 0; v < 4; v++) {
                    double ur = sr_[rb][v], ui = si_[rb][v];
                    if (PLAIN) {
                        const bool piv = ztile_row<RPW>(w, rb, l, v) == j;
                        const double t0 = scr * ur - sci * ui;
                        ui = piv ? 0.0 : scr * ui + sci * ur;
                        ur = piv ? 1.0 : t0;
                    }
                    xr[rb][ct][v] -= ur * kr - ui * ki;
                    xi[rb][ct][v] -= ur * ki + ui * kr;
                }
        }
        if (PLAIN && cl == clj) {
#pragma unroll
            for (int rb = 0; rb < RB; rb++)
#pragma unroll
                for (int v = 0; v < 4; v++)
                    if (ztile_row<RPW>(w, rb, l, v) == j) {
                        xr[rb][CTJ][v] = beta;
                        xi[rb][CTJ][v] = 0.0;
                    }
        }
        cy.beta_prev = beta;
    }
}

template <int KP, bool PLAIN>
__device__ __forceinline__ double zhh_tile(d4 (&xr)[ZGeo<KP>::RB][KP / 16], d4 (&xi)[ZGeo<KP>::RB][KP / 16], int k,
                                           int w, const ZShm& S) {
    constexpr int RB = ZGeo<KP>::RB, RPW = ZGeo<KP>::RPW, CT = KP / 16;
    ZCarry cy = {0.0, 0.0, 0.0, 0.0, 0.0};
    zhh_block<KP, PLAIN, 0>(xr, xi, k, w, S, cy);
    if constexpr (CT > 1) zhh_block<KP, PLAIN, 1>(xr, xi, k, w, S, cy);
    // the Householder vectors: column c = 16 ct + l % 16 times its s_c (0
    // for padding columns and tau = 0 columns, whose sub-columns are zero)
    double mr[4], mi[4];
    gather_cols(cy.msr, mr);
    gather_cols(cy.msi, mi);
    const int l = zlane(), cl = l & 15;
#pragma unroll
    for (int rb = 0; rb < RB; rb++)
#pragma unroll
        for (int ct = 0; ct < CT; ct++)
#pragma unroll
            for (int v = 0; v < 4; v++) {
                if (!PLAIN || ztile_row<RPW>(w, rb, l, v) > 16 * ct + cl) {
                    const double a = xr[rb][ct][v], b = xi[rb][ct][v];
                    xr[rb][ct][v] = a * mr[ct] - b * mi[ct];
                    xi[rb][ct][v] = a * mi[ct] + b * mr[ct];
                }
            }
    return cy.beta_prev;
}

// acr + i aci += X[rows, :] B over the rows row0 + 16 rb + (0..15) of a full
// tile (every row present, all 4 KS columns valid): X complex row-major (ld
// ldx, in doubles of pairs), K index 4 s + lane / 16 (two K-steps read a
// whole 128-byte line of each row), B complex in B-operand order
// (k_zpermute_b), four real MFMA products per complex one.  Batches of two
// K-steps; the loads of the next batch are issued before the MFMAs of the
// current one.
template <int RB, int CT, int KS>
__device__ __forceinline__ void zprod_full(d4 (&acr)[RB][CT], d4 (&aci)[RB][CT], const double* __restrict__ X,
                                           int ldx, int row0, const double* __restrict__ B, int l) {
    constexpr int SC = 2, NBT = KS / SC;
    static_assert(NBT * SC == KS, "KS must be even");
    const int g = l >> 4, cl = l & 15;
    auto load = [&](int s0, double2(&a)[RB][SC], double2(&b)[SC][CT]) {
#pragma unroll
        for (int rb = 0; rb < RB; rb++) {
            const double* xr = X + 2 * (row0 + 16 * rb + cl) * ldx;
#pragma unroll
            for (int s = 0; s < SC; s++) a[rb][s] = ld2(xr + 2 * (4 * (s0 + s) + g));
        }
#pragma unroll
        for (int s = 0; s < SC; s++)
#pragma unroll
            for (int ct = 0; ct < CT; ct++) b[s][ct] = ld2(B + 2 * (((s0 + s) * CT + ct) * 64 + l));
    };
    double2 a[2][RB][SC], b[2][SC][CT];
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
                for (int ct = 0; ct < CT; ct++) {
                    const double2 x = a[cur][rb][s], y = b[cur][s][ct];
                    acr[rb][ct] = mfma(x.x, y.x, acr[rb][ct]);
                    acr[rb][ct] = mfma(-x.y, y.y, acr[rb][ct]);
                    aci[rb][ct] = mfma(x.x, y.y, aci[rb][ct]);
                    aci[rb][ct] = mfma(x.y, y.x, aci[rb][ct]);
                }
    }
}

template <int KP, int K0P>
__global__ __launch_bounds__(ZNW * 64, 2) void k_zleaf_rt(ZRLevel L) {
    constexpr int RB = ZGeo<KP>::RB, RPW = ZGeo<KP>::RPW, TB = ZGeo<KP>::TB, CT = KP / 16, LDT = KP + 1;
    constexpr bool HASV = K0P > 0;
    constexpr int KS0 = HASV ? K0P / 4 : 1;
    constexpr int MT0 = HASV ? K0P / 16 : 1;
    constexpr int NJW = (MT0 + ZNW - 1) / ZNW;

    extern __shared__ double sm[];
    ZShm S;
    S.sr = sm;
    S.si = S.sr + KP * LDT;
    S.gr = S.si + KP * LDT;
    S.gi = S.gr + KP * LDT;
    S.tlr = S.gi + KP * LDT;
    S.tli = S.tlr + KP * LDT;
    S.xr = S.tli + KP * LDT;
    S.xi = S.xr + TB;
    S.prr = S.xi + TB;
    S.pri = S.prr + 2 * KP;
    S.ptr = S.pri + 2 * KP;
    S.pti = S.ptr + 2 * ZNW * KP;
    S.tar = S.pti + 2 * ZNW * KP;
    S.tai = S.tar + KP;

    const int c = blockIdx.x;
    const int tid = threadIdx.x, w = tid >> 6;
    const int k = L.k;
    const int k0 = HASV ? L.k0 : 0;
    const int64_t cr0 = (int64_t)c * L.m / L.nchunk;
    const int64_t cr1 = (int64_t)(c + 1) * L.m / L.nchunk;
    const int ntiles = (int)((cr1 - cr0 + TB - 1) / TB);
    double* NT = HASV ? (double*)(L.Nc + (int64_t)c * KP * K0P) : nullptr;  // M_c (KP x K0P complex)

    for (int t = 0; t < ntiles; t++) {
        if (t > 0) __syncthreads();
        const int64_t r0 = cr0 + (int64_t)t * TB;
        const int trows = (int)((cr1 - r0 < TB) ? (cr1 - r0) : TB);
        const bool plain = (t == 0);
        const double* __restrict__ Xt = (const double*)(L.X + r0 * L.ldx);
        double* __restrict__ Yt = (double*)(L.Y + r0 * L.ldy);
        const double* __restrict__ Vt = HASV ? (const double*)(L.V + r0 * L.ldv) : nullptr;
        const int ldx = (int)L.ldx, ldy = (int)L.ldy, ldv = (int)L.ldv;

        d4 xr[RB][CT], xi[RB][CT];
        {
            const int l = zlane(), cl = l & 15;
#pragma unroll
            for (int rb = 0; rb < RB; rb++)
#pragma unroll
                for (int ct = 0; ct < CT; ct++)
#pragma unroll
                    for (int v = 0; v < 4; v++) {
                        const int row = ztile_row<RPW>(w, rb, l, v), col = 16 * ct + cl;
                        double2 z = make_double2(0.0, 0.0);
                        if (row < trows && col < k) z = ld2(Xt + 2 * (row * ldx + col));
                        xr[rb][ct][v] = z.x;
                        xi[rb][ct][v] = z.y;
                    }
        }
        // A <- A + V Z (four real MFMA products per complex one; Z in
        // B-operand order, k_zpermute_b)
        if (HASV && k0 > 0) {
            // a full tile takes the unmasked, pipelined product
            const bool fullv = trows == TB && k0 == K0P;
            if constexpr (HASV) {
                if (fullv) zprod_full<RB, CT, KS0>(xr, xi, Vt, ldv, RPW * w, (const double*)L.Zp, zlane());
            }
            const int l = zlane(), g = l >> 4, cl = l & 15;
            constexpr int SC = 2;
#pragma unroll 2
            for (int s0 = 0; s0 < (fullv ? 0 : KS0); s0 += SC) {
                double ar_[RB][SC], ai_[RB][SC], br_[SC][CT], bi_[SC][CT];
#pragma unroll
                for (int rb = 0; rb < RB; rb++) {
                    const int vr = RPW * w + 16 * rb + cl;
#pragma unroll
                    for (int s = 0; s < SC; s++) {
                        const int kk = 4 * (s0 + s) + g;  // a K-step pair reads whole lines of V
                        double2 z = make_double2(0.0, 0.0);
                        if (vr < trows && kk < k0) z = ld2(Vt + 2 * (vr * ldv + kk));
                        ar_[rb][s] = z.x;
                        ai_[rb][s] = z.y;
                    }
                }
#pragma unroll
                for (int s = 0; s < SC; s++)
#pragma unroll
                    for (int ct = 0; ct < CT; ct++) {
                        const double2 z = ld2((const double*)L.Zp + 2 * (((s0 + s) * CT + ct) * 64 + l));
                        br_[s][ct] = z.x;
                        bi_[s][ct] = z.y;
                    }
#pragma unroll
                for (int s = 0; s < SC; s++)
#pragma unroll
                    for (int rb = 0; rb < RB; rb++)
#pragma unroll
                        for (int ct = 0; ct < CT; ct++) {
                            xr[rb][ct] = mfma(ar_[rb][s], br_[s][ct], xr[rb][ct]);
                            xr[rb][ct] = mfma(-ai_[rb][s], bi_[s][ct], xr[rb][ct]);
                            xi[rb][ct] = mfma(ar_[rb][s], bi_[s][ct], xi[rb][ct]);
                            xi[rb][ct] = mfma(ai_[rb][s], br_[s][ct], xi[rb][ct]);
                        }
            }
        }

        double beta_last;
        if (plain) beta_last = zhh_tile<KP, true>(xr, xi, k, w, S);
        else beta_last = zhh_tile<KP, false>(xr, xi, k, w, S);
        __syncthreads();
        if (!plain && w == 0 && k > 0 && (threadIdx.x & 63) == k - 1) {
            S.sr[(k - 1) * LDT + (k - 1)] = beta_last;
            S.si[(k - 1) * LDT + (k - 1)] = 0.0;
        }
        {
            const int l = zlane(), cl = l & 15;
            if (plain) {
                // R -> slot; registers -> U_0 (explicit unit diagonal, zeros above)
#pragma unroll
                for (int rb = 0; rb < RB; rb++)
#pragma unroll
                    for (int ct = 0; ct < CT; ct++)
#pragma unroll
                        for (int v = 0; v < 4; v++) {
                            const int row = ztile_row<RPW>(w, rb, l, v), col = 16 * ct + cl;
                            if (row < KP && col < KP) {
                                const bool up = col >= row && row < k && col < k;
                                S.sr[row * LDT + col] = up ? xr[rb][ct][v] : 0.0;
                                S.si[row * LDT + col] = up ? xi[rb][ct][v] : 0.0;
                                if (col > row) {
                                    xr[rb][ct][v] = 0.0;
                                    xi[rb][ct][v] = 0.0;
                                } else if (col == row) {
                                    xr[rb][ct][v] = (row < k) ? 1.0 : 0.0;
                                    xi[rb][ct][v] = 0.0;
                                }
                            }
                        }
            }
#pragma unroll
            for (int rb = 0; rb < RB; rb++)
#pragma unroll
                for (int ct = 0; ct < CT; ct++)
#pragma unroll
                    for (int v = 0; v < 4; v++) {
                        const int row = ztile_row<RPW>(w, rb, l, v), col = 16 * ct + cl;
                        if (row < trows && col < k) st2(Yt + 2 * (row * ldy + col), xr[rb][ct][v], xi[rb][ct][v]);
                    }
        }
        // T factor (H_0 ... H_{k-1} = I - U T U^H) in 16 x 16 blocks: each
        // diagonal block by the recurrence T(r, r) = tau_r,
        // T(r, i) = -tau_i sum_{r <= p < i} T(r, p) G(p, i) within the block
        // (one thread per row, the blocks in parallel); then, for KP = 32,
        // the off-diagonal block X = -T_a (U_a^H U_b) T_b of the product of
        // the two blocks' transformations
        if (tid < KP) {
            const int r = tid, b0 = (r / 16) * 16;
            double Trr[16], Tri[16];  // T(r, b0 + jj)
#pragma unroll
            for (int jj = 0; jj < 16; jj++) {
                Trr[jj] = (b0 + jj == r && r < k) ? S.tar[r] : 0.0;
                Tri[jj] = (b0 + jj == r && r < k) ? S.tai[r] : 0.0;
            }
#pragma unroll
            for (int ii = 1; ii < 16; ii++) {
                const int i = b0 + ii;
                if (i > r && i < k) {
                    double sr2 = 0.0, si2 = 0.0;
#pragma unroll
                    for (int pp = 0; pp < ii; pp++)
                        if (b0 + pp >= r) {
                            const double gr = S.gr[i * LDT + b0 + pp], gi = S.gi[i * LDT + b0 + pp];
                            sr2 += Trr[pp] * gr - Tri[pp] * gi;
                            si2 += Trr[pp] * gi + Tri[pp] * gr;
                        }
                    const double tr = S.tar[i], ti = S.tai[i];
                    Trr[ii] = -(tr * sr2 - ti * si2);
                    Tri[ii] = -(tr * si2 + ti * sr2);
                }
            }
#pragma unroll
            for (int jj = 0; jj < 16; jj++) {
                S.tlr[r * LDT + b0 + jj] = Trr[jj];
                S.tli[r * LDT + b0 + jj] = Tri[jj];
            }
            if constexpr (KP == 32) {
                // the other block of row r: zero below the diagonal blocks
                // (block b, row r >= 16); block a rows are overwritten by X
                const int o0 = 16 - b0;
#pragma unroll
                for (int jj = 0; jj < 16; jj++) {
                    S.tlr[r * LDT + o0 + jj] = 0.0;
                    S.tli[r * LDT + o0 + jj] = 0.0;
                }
            }
        }
        if constexpr (KP == 32) {
            __syncthreads();
            // Y1 = G_ab T_b (16 x 16), G(p, q) at [q][p]; kept in the unused
            // upper part of the Gram array, Y1(p, i) at [p][i] (p < 16 <= i)
            {
                const int p = tid >> 4, i = 16 + (tid & 15);
                double yr = 0.0, yi = 0.0;
                for (int q = 16; q <= i; q++) {
                    const double gr = S.gr[q * LDT + p], gi = S.gi[q * LDT + p];
                    const double tr = S.tlr[q * LDT + i], ti = S.tli[q * LDT + i];
                    yr += gr * tr - gi * ti;
                    yi += gr * ti + gi * tr;
                }
                S.gr[p * LDT + i] = yr;
                S.gi[p * LDT + i] = yi;
            }
            __syncthreads();
            // X(r, i) = -sum_{r <= p < 16} T_a(r, p) Y1(p, i)
            {
                const int r = tid >> 4, i = 16 + (tid & 15);
                double xr2 = 0.0, xi2 = 0.0;
                for (int p = r; p < 16; p++) {
                    const double tr = S.tlr[r * LDT + p], ti = S.tli[r * LDT + p];
                    const double yr = S.gr[p * LDT + i], yi = S.gi[p * LDT + i];
                    xr2 += tr * yr - ti * yi;
                    xi2 += tr * yi + ti * yr;
                }
                S.tlr[r * LDT + i] = (r < k && i < k) ? -xr2 : 0.0;
                S.tli[r * LDT + i] = (r < k && i < k) ? -xi2 : 0.0;
            }
        }
        __syncthreads();
        {
            double* Tg = (double*)(L.Tt + ((int64_t)c * L.maxtiles + t) * KP * KP);
            for (int e = tid; e < KP * KP; e += blockDim.x) {
                const int r = e / KP, jj = e % KP;
                st2(Tg + 2 * e, S.tlr[r * LDT + jj], S.tli[r * LDT + jj]);
            }
        }
        __syncthreads();  // T is in LDS; every read of the Gram is done
        if (HASV && k0 > 0) {
            const int l = zlane(), g = l >> 4, cl = l & 15;
            // S = M + Y^H V (structured) or Y^H V (plain)
            d4 ar[CT][NJW], ai[CT][NJW];
#pragma unroll
            for (int mi = 0; mi < CT; mi++)
#pragma unroll
                for (int q = 0; q < NJW; q++)
#pragma unroll
                    for (int v = 0; v < 4; v++) {
                        const int rr = 16 * mi + drow(l, v), cc = 16 * (w + ZNW * q) + cl;
                        double2 z = make_double2(0.0, 0.0);
                        if (!plain && cc < K0P) z = ld2(NT + 2 * (rr * K0P + cc));
                        ar[mi][q][v] = z.x;
                        ai[mi][q][v] = z.y;
                    }
            constexpr int US = 2;
            for (int s0 = 0; s0 < TB / 4; s0 += US) {
                double yr[US][CT], yi[US][CT], vr_[US][NJW], vi_[US][NJW];
#pragma unroll
                for (int u = 0; u < US; u++) {
                    const int row = 4 * (s0 + u) + g;
                    const bool ok = row < trows;
#pragma unroll
                    for (int mi = 0; mi < CT; mi++) {
                        const int yc = 16 * mi + cl;
                        double2 z = make_double2(0.0, 0.0);
                        if (ok && yc < k) z = ld2(Yt + 2 * (row * ldy + yc));
                        yr[u][mi] = z.x;
                        yi[u][mi] = z.y;
                    }
#pragma unroll
                    for (int q = 0; q < NJW; q++) {
                        const int vc = 16 * (w + ZNW * q) + cl;
                        double2 z = make_double2(0.0, 0.0);
                        if (ok && vc < k0) z = ld2(Vt + 2 * (row * ldv + vc));
                        vr_[u][q] = z.x;
                        vi_[u][q] = z.y;
                    }
                }
                // conj(y) v = (yr vr + yi vi) + i (yr vi - yi vr)
#pragma unroll
                for (int u = 0; u < US; u++)
#pragma unroll
                    for (int mi = 0; mi < CT; mi++)
#pragma unroll
                        for (int q = 0; q < NJW; q++) {
                            ar[mi][q] = mfma(yr[u][mi], vr_[u][q], ar[mi][q]);
                            ar[mi][q] = mfma(yi[u][mi], vi_[u][q], ar[mi][q]);
                            ai[mi][q] = mfma(yr[u][mi], vi_[u][q], ai[mi][q]);
                            ai[mi][q] = mfma(-yi[u][mi], vr_[u][q], ai[mi][q]);
                        }
            }
            // D = T^H S: (T^H)(m, p) = conj(T(p, m)), K-step (rb, v) takes the
            // rows 16 rb + l/16 + 4 v of S (register v of block rb)
            d4 dr[CT][NJW], di[CT][NJW];
#pragma unroll
            for (int mi = 0; mi < CT; mi++)
#pragma unroll
                for (int q = 0; q < NJW; q++) dr[mi][q] = di[mi][q] = d4zero();
#pragma unroll
            for (int rb = 0; rb < CT; rb++)
#pragma unroll
                for (int v = 0; v < 4; v++) {
                    const int p = 16 * rb + drow(l, v);
#pragma unroll
                    for (int mi = 0; mi < CT; mi++) {
                        if (rb > mi) continue;  // T^H is lower triangular
                        const int m = 16 * mi + cl;
                        const double tr = S.tlr[p * LDT + m], ti = -S.tli[p * LDT + m];
#pragma unroll
                        for (int q = 0; q < NJW; q++) {
                            dr[mi][q] = mfma(tr, ar[rb][q][v], dr[mi][q]);
                            dr[mi][q] = mfma(-ti, ai[rb][q][v], dr[mi][q]);
                            di[mi][q] = mfma(tr, ai[rb][q][v], di[mi][q]);
                            di[mi][q] = mfma(ti, ar[rb][q][v], di[mi][q]);
                        }
                    }
                }
            if (!plain) {
#pragma unroll
                for (int mi = 0; mi < CT; mi++)
#pragma unroll
                    for (int q = 0; q < NJW; q++)
#pragma unroll
                        for (int v = 0; v < 4; v++) {
                            const int rr = 16 * mi + drow(l, v), cc = 16 * (w + ZNW * q) + cl;
                            if (cc < K0P) {
                                double* pz = NT + 2 * (rr * K0P + cc);
                                const double2 z = ld2(pz);
                                st2(pz, z.x - dr[mi][q][v], z.y - di[mi][q][v]);
                            }
                        }
            } else {
                // E = L_0 D, L_0 = Y_0[0:k, 0:k] (unit lower); M = V_0[0:k] - E
                d4 er[CT][NJW], ei[CT][NJW];
#pragma unroll
                for (int mi = 0; mi < CT; mi++)
#pragma unroll
                    for (int q = 0; q < NJW; q++) er[mi][q] = ei[mi][q] = d4zero();
#pragma unroll
                for (int rb = 0; rb < CT; rb++)
#pragma unroll
                    for (int v = 0; v < 4; v++) {
                        const int p = 16 * rb + drow(l, v);
#pragma unroll
                        for (int mi = 0; mi < CT; mi++) {
                            if (rb > mi) continue;
                            const int m = 16 * mi + cl;
                            double2 z = make_double2(0.0, 0.0);
                            if (m < k && p < k) z = ld2(Yt + 2 * (m * ldy + p));
#pragma unroll
                            for (int q = 0; q < NJW; q++) {
                                er[mi][q] = mfma(z.x, dr[rb][q][v], er[mi][q]);
                                er[mi][q] = mfma(-z.y, di[rb][q][v], er[mi][q]);
                                ei[mi][q] = mfma(z.x, di[rb][q][v], ei[mi][q]);
                                ei[mi][q] = mfma(z.y, dr[rb][q][v], ei[mi][q]);
                            }
                        }
                    }
#pragma unroll
                for (int mi = 0; mi < CT; mi++)
#pragma unroll
                    for (int q = 0; q < NJW; q++)
#pragma unroll
                        for (int v = 0; v < 4; v++) {
                            const int rr = 16 * mi + drow(l, v), cc = 16 * (w + ZNW * q) + cl;
                            double2 z = make_double2(0.0, 0.0);
                            if (rr < k && cc < k0) z = ld2(Vt + 2 * (rr * ldv + cc));
                            if (cc < K0P) st2(NT + 2 * (rr * K0P + cc), z.x - er[mi][q][v], z.y - ei[mi][q][v]);
                        }
            }
        }
    }
    __syncthreads();
    for (int e = tid; e < k * KP; e += blockDim.x) {
        const int i = e / KP, jj = e % KP;
        const bool up = jj < k && jj >= i;
        st2((double*)(L.Rnext + ((int64_t)c * k + i) * L.ldrn + jj), up ? S.sr[i * LDT + jj] : 0.0,
            up ? S.si[i * LDT + jj] : 0.0);
    }
}

// Z (k0 x k complex, ld ldz) into the B-operand order of the fused update:
// entry ((s * CT + ct) * 64 + l) holds Z[4 s + l / 16][16 ct + l % 16] (the
// four lane groups take adjacent K indices, so that two K-steps read whole
// 128-byte lines of the streamed rows), zero outside k0 x k.
__global__ void k_zpermute_b(int k0p, int kp, int k0, int k, const dcplx* __restrict__ Z, int64_t ldz, dcplx* out) {
    const int ks = k0p / 4, ct_n = kp / 16;
    const int total = ks * ct_n * 64;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
        const int l = e & 63, sct = e >> 6;
        const int s = sct / ct_n, ct = sct % ct_n;
        const int r = 4 * s + (l >> 4), cc = 16 * ct + (l & 15);
        out[e] = (r < k0 && cc < k) ? Z[(int64_t)r * ldz + cc] : dcplx{0.0, 0.0};
    }
}

// Per chunk, out_c = M_c^H G_c (k0 x k complex, ld kp): M_c the chunk's
// Q_chunk^H V_chunk (KP x K0P), G_c the chunk's block of the formed Q of the
// level above (rows c * gstride .., ld ldg); both staged through LDS.
__global__ void k_zchunk_prod(int k0, int k, int kp, int k0p, const dcplx* __restrict__ M,
                              const dcplx* __restrict__ G, int64_t ldg, int64_t gstride, dcplx* out) {
    extern __shared__ double sm[];
    dcplx* Ms = (dcplx*)sm;   // kp x k0p
    dcplx* Gs = Ms + kp * k0p;  // kp x kp
    const int c = blockIdx.x;
    const dcplx* Mc = M + (int64_t)c * kp * k0p;
    const dcplx* Gc = G + (int64_t)c * gstride * ldg;
    dcplx* Oc = out + (int64_t)c * k0p * kp;
    for (int e = threadIdx.x; e < kp * k0p; e += blockDim.x) Ms[e] = Mc[e];
    for (int e = threadIdx.x; e < kp * kp; e += blockDim.x) {
        const int p = e / kp, j = e % kp;
        Gs[e] = (p < k && j < k) ? Gc[(int64_t)p * ldg + j] : dcplx{0.0, 0.0};
    }
    __syncthreads();
    for (int e = threadIdx.x; e < k0p * kp; e += blockDim.x) {
        const int i = e / kp, j = e % kp;
        double sr = 0.0, si = 0.0;
        if (i < k0 && j < k)
            for (int p = 0; p < k; p++) {
                const dcplx a = Ms[p * k0p + i], b = Gs[p * kp + j];
                sr += a.re * b.re + a.im * b.im;  // conj(a) b
                si += a.re * b.im - a.im * b.re;
            }
        Oc[e] = dcplx{sr, si};
    }
}

// ---------------------------------------------------------------------------
// Formation of level 0 in two passes, as in the real path: per chunk the
// k x k recurrence top-down (K_t = T_t C, C <- C - K_t for a structured
// tile; K_0 = T_0 U_0[0:k]^H C for tile 0, whose top k rows also receive
// C), with -K_t written over T_t in B-operand order and the final C into
// Cfin; then every tile on its own: Q_t = [C; 0] (tile 0) - Y_t K_t + V_t N.

template <int KP>
__global__ __launch_bounds__(256) void k_zkchain(ZLevel L, dcplx* Cfin) {
    constexpr int LD = KP + 1, KS = KP / 4, CT = KP / 16;
    constexpr int TB = ZGeo<KP>::TB;
    extern __shared__ double sm[];
    dcplx* Cs = (dcplx*)sm;    // KP x LD: the running C
    dcplx* Es = Cs + KP * LD;  // KP x LD
    dcplx* Ts = Es + KP * LD;  // KP x LD: T_t
    const int tid = threadIdx.x, c = blockIdx.x, k = L.k;
    const int64_t cr0 = (int64_t)c * L.m / L.nchunk;
    const int64_t cr1 = (int64_t)(c + 1) * L.m / L.nchunk;
    const int ntiles = (int)((cr1 - cr0 + TB - 1) / TB);
    {
        const dcplx* G = L.Gin + (int64_t)c * L.gstride * L.ldg;
        for (int e = tid; e < KP * KP; e += blockDim.x) {
            const int i = e / KP, j = e % KP;
            Cs[i * LD + j] = (i < k && j < k) ? G[(int64_t)i * L.ldg + j] : dcplx{0.0, 0.0};
        }
    }
    const dcplx* Y0 = L.Y + cr0 * L.ldy;
    for (int t = ntiles - 1; t >= 0; t--) {
        const bool plain = (t == 0);
        dcplx* Tt = L.Tt + ((int64_t)c * L.maxtiles + t) * KP * KP;
        __syncthreads();
        for (int e = tid; e < KP * KP; e += blockDim.x) Ts[(e / KP) * LD + e % KP] = Tt[e];
        // E = U_0[0:k]^H C (tile 0) or C
        for (int e = tid; e < KP * KP; e += blockDim.x) {
            const int i = e / KP, j = e % KP;
            double sr = 0.0, si = 0.0;
            if (i < k && j < k) {
                if (plain) {
                    for (int p = 0; p < k; p++) {
                        const dcplx a = Y0[(int64_t)p * L.ldy + i], b = Cs[p * LD + j];
                        sr += a.re * b.re + a.im * b.im;
                        si += a.re * b.im - a.im * b.re;
                    }
                } else {
                    sr = Cs[i * LD + j].re;
                    si = Cs[i * LD + j].im;
                }
            }
            Es[i * LD + j] = dcplx{sr, si};
        }
        __syncthreads();
        // K = T E (T upper triangular); -K over T_t in B-operand order
        for (int e = tid; e < KP * KP; e += blockDim.x) {
            const int i = e / KP, j = e % KP;
            double sr = 0.0, si = 0.0;
            if (i < k && j < k)
                for (int p = i; p < k; p++) {
                    const dcplx a = Ts[i * LD + p], b = Es[p * LD + j];
                    sr += a.re * b.re - a.im * b.im;
                    si += a.re * b.im + a.im * b.re;
                }
            // row i of K is K-step i / 4 of lane group i % 4 (the split of zprod_full)
            Tt[((i >> 2) * CT + j / 16) * 64 + 16 * (i & 3) + (j % 16)] = dcplx{-sr, -si};
            if (!plain) Cs[i * LD + j] = dcplx{Cs[i * LD + j].re - sr, Cs[i * LD + j].im - si};
        }
    }
    __syncthreads();
    dcplx* Cf = Cfin + (int64_t)c * KP * KP;
    for (int e = tid; e < KP * KP; e += blockDim.x) Cf[e] = Cs[(e / KP) * LD + e % KP];
}

// One workgroup per tile slot: Q_t = [C; 0] (tile 0) - Y_t K_t + V_t N on
// MFMA (four real products per complex one), in place of Y_t; every
// wavefront reads and writes only its own rows.
template <int KP, int K0P>
__global__ __launch_bounds__(ZNW * 64, 2) void k_zrows(ZLevel L, const dcplx* Cfin, const dcplx* V, int64_t ldv,
                                                      int k0, const dcplx* Np) {
    constexpr int RB = ZGeo<KP>::RB, RPW = ZGeo<KP>::RPW, TB = ZGeo<KP>::TB, CT = KP / 16, KS = KP / 4;
    constexpr int KS0 = K0P > 0 ? K0P / 4 : 1;
    const int c = blockIdx.x / L.maxtiles, t = blockIdx.x % L.maxtiles;
    const int w = threadIdx.x >> 6, k = L.k;
    const int64_t cr0 = (int64_t)c * L.m / L.nchunk;
    const int64_t cr1 = (int64_t)(c + 1) * L.m / L.nchunk;
    const int64_t r0 = cr0 + (int64_t)t * TB;
    if (r0 >= cr1) return;  // slot beyond this chunk's tiles (uniform)
    const int trows = (int)((cr1 - r0 < TB) ? (cr1 - r0) : TB);
    const double* Kg = (const double*)(L.Tt + ((int64_t)c * L.maxtiles + t) * KP * KP);  // -K_t
    double* Yt = (double*)(L.Y + r0 * L.ldy);
    const int ldy = (int)L.ldy;
    const int l = lane_id(), g = l >> 4, cl = l & 15;
    d4 acr[RB][CT], aci[RB][CT];
#pragma unroll
    for (int rb = 0; rb < RB; rb++)
#pragma unroll
        for (int ct = 0; ct < CT; ct++) {
            acr[rb][ct] = d4zero();
            aci[rb][ct] = d4zero();
        }
    if (t == 0) {
        const double* Cf = (const double*)(Cfin + (int64_t)c * KP * KP);
#pragma unroll
        for (int rb = 0; rb < RB; rb++)
#pragma unroll
            for (int ct = 0; ct < CT; ct++)
#pragma unroll
                for (int v = 0; v < 4; v++) {
                    const int row = ztile_row<RPW>(w, rb, l, v), col = 16 * ct + cl;
                    if (row < KP) {
                        const double2 z = ld2(Cf + 2 * (row * KP + col));
                        acr[rb][ct][v] = z.x;
                        aci[rb][ct][v] = z.y;
                    }
                }
    }
    // - Y_t K_t (the stored -K_t, K split 4 s + lane / 16)
    const bool fullk = trows == TB && k == KP;
    if (fullk) zprod_full<RB, CT, KS>(acr, aci, Yt, ldy, RPW * w, Kg, l);
    else
#pragma unroll
    for (int rb = 0; rb < RB; rb++) {
        const int yr = RPW * w + 16 * rb + cl;
        double ar[KS], ai[KS];
#pragma unroll
        for (int s = 0; s < KS; s++) {
            double2 z = make_double2(0.0, 0.0);
            if (yr < trows && 4 * s + g < k) z = ld2(Yt + 2 * (yr * ldy + 4 * s + g));
            ar[s] = z.x;
            ai[s] = z.y;
        }
#pragma unroll
        for (int s = 0; s < KS; s++)
#pragma unroll
            for (int ct = 0; ct < CT; ct++) {
                const double2 b = ld2(Kg + 2 * ((s * CT + ct) * 64 + l));
                acr[rb][ct] = mfma(ar[s], b.x, acr[rb][ct]);
                acr[rb][ct] = mfma(-ai[s], b.y, acr[rb][ct]);
                aci[rb][ct] = mfma(ar[s], b.y, aci[rb][ct]);
                aci[rb][ct] = mfma(ai[s], b.x, aci[rb][ct]);
            }
    }
    // + V_t N (N in B-operand order)
    if (K0P > 0 && k0 > 0) {
        const double* Vt = (const double*)(V + r0 * ldv);
        const bool fullv = trows == TB && k0 == K0P;
        if constexpr (K0P > 0) {
            if (fullv) zprod_full<RB, CT, KS0>(acr, aci, Vt, (int)ldv, RPW * w, (const double*)Np, l);
        }
        constexpr int SC = 4;
#pragma unroll 2
        for (int s0 = 0; s0 < (fullv ? 0 : KS0); s0 += SC) {
            double vr[RB][SC], vi[RB][SC], br[SC][CT], bi[SC][CT];
#pragma unroll
            for (int rb = 0; rb < RB; rb++) {
                const int xr = RPW * w + 16 * rb + cl;
#pragma unroll
                for (int s = 0; s < SC; s++) {
                    const int kk = 4 * (s0 + s) + g;
                    double2 z = make_double2(0.0, 0.0);
                    if (xr < trows && kk < k0) z = ld2(Vt + 2 * (xr * ldv + kk));
                    vr[rb][s] = z.x;
                    vi[rb][s] = z.y;
                }
            }
#pragma unroll
            for (int s = 0; s < SC; s++)
#pragma unroll
                for (int ct = 0; ct < CT; ct++) {
                    const double2 z = ld2((const double*)Np + 2 * (((s0 + s) * CT + ct) * 64 + l));
                    br[s][ct] = z.x;
                    bi[s][ct] = z.y;
                }
#pragma unroll
            for (int s = 0; s < SC; s++)
#pragma unroll
                for (int rb = 0; rb < RB; rb++)
#pragma unroll
                    for (int ct = 0; ct < CT; ct++) {
                        acr[rb][ct] = mfma(vr[rb][s], br[s][ct], acr[rb][ct]);
                        acr[rb][ct] = mfma(-vi[rb][s], bi[s][ct], acr[rb][ct]);
                        aci[rb][ct] = mfma(vr[rb][s], bi[s][ct], aci[rb][ct]);
                        aci[rb][ct] = mfma(vi[rb][s], br[s][ct], aci[rb][ct]);
                    }
        }
    }
#pragma unroll
    for (int rb = 0; rb < RB; rb++)
#pragma unroll
        for (int ct = 0; ct < CT; ct++)
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int row = ztile_row<RPW>(w, rb, l, v), col = 16 * ct + cl;
                if (row < trows && col < k) st2(Yt + 2 * (row * ldy + col), acr[rb][ct][v], aci[rb][ct][v]);
            }
}

template <int KP>
hipError_t zkchain_t(const ZLevel& L, dcplx* Cfin, hipStream_t st) {
    const size_t shm = 3 * KP * (KP + 1) * sizeof(dcplx);
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void*)k_zkchain<KP>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)shm);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL((k_zkchain<KP>), dim3(L.nchunk), dim3(256), shm, st, L, Cfin);
    return hipGetLastError();
}

template <int KP, int K0P>
hipError_t zrows_t(const ZLevel& L, const dcplx* Cfin, const dcplx* V, int64_t ldv, int k0, const dcplx* Np,
                   hipStream_t st) {
    hipLaunchKernelGGL((k_zrows<KP, K0P>), dim3((int64_t)L.nchunk * L.maxtiles), dim3(ZNW * 64), 0, st, L, Cfin, V,
                       ldv, k0, Np);
    return hipGetLastError();
}

template <int KP, int K0P>
hipError_t zleaf_rt_t(const ZRLevel& L, hipStream_t st) {
    const size_t shm = ZLeafLds<KP>::total * sizeof(double);
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void*)k_zleaf_rt<KP, K0P>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)shm);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL((k_zleaf_rt<KP, K0P>), dim3(L.nchunk), dim3(ZNW * 64), shm, st, L);
    return hipGetLastError();
}

}  // namespace

int zleaf_rt_tile_rows(int kp) { return kp <= 16 ? ZGeo<16>::TB : ZGeo<32>::TB; }

hipError_t launch_zleaf_rt(int kp, int k0p, const ZRLevel& L, hipStream_t st) {
    if (k0p > 0 && (L.V == nullptr || L.Zp == nullptr || L.Nc == nullptr)) return hipErrorInvalidValue;
    switch (kp * 1000 + k0p) {
        case 16000: return zleaf_rt_t<16, 0>(L, st);
        case 16016: return zleaf_rt_t<16, 16>(L, st);
        case 16032: return zleaf_rt_t<16, 32>(L, st);
        case 16064: return zleaf_rt_t<16, 64>(L, st);
        case 32000: return zleaf_rt_t<32, 0>(L, st);
        case 32016: return zleaf_rt_t<32, 16>(L, st);
        case 32032: return zleaf_rt_t<32, 32>(L, st);
        case 32064: return zleaf_rt_t<32, 64>(L, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_zkchain(int kp, const ZLevel& L, dcplx* Cfin, hipStream_t st) {
    if (kp == 16) return zkchain_t<16>(L, Cfin, st);
    if (kp == 32) return zkchain_t<32>(L, Cfin, st);
    return hipErrorInvalidValue;
}

hipError_t launch_zrows0(int kp, int k0p, const ZLevel& L, const dcplx* Cfin, const dcplx* V, int64_t ldv, int k0,
                         const dcplx* Np, hipStream_t st) {
    switch (kp * 1000 + k0p) {
        case 16000: return zrows_t<16, 0>(L, Cfin, V, ldv, k0, Np, st);
        case 16016: return zrows_t<16, 16>(L, Cfin, V, ldv, k0, Np, st);
        case 16032: return zrows_t<16, 32>(L, Cfin, V, ldv, k0, Np, st);
        case 16064: return zrows_t<16, 64>(L, Cfin, V, ldv, k0, Np, st);
        case 32000: return zrows_t<32, 0>(L, Cfin, V, ldv, k0, Np, st);
        case 32016: return zrows_t<32, 16>(L, Cfin, V, ldv, k0, Np, st);
        case 32032: return zrows_t<32, 32>(L, Cfin, V, ldv, k0, Np, st);
        case 32064: return zrows_t<32, 64>(L, Cfin, V, ldv, k0, Np, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_zpermute_b(int k0p, int kp, int k0, int k, const dcplx* Z, int64_t ldz, dcplx* out, hipStream_t st) {
    const int total = (k0p / 4) * (kp / 16) * 64;
    hipLaunchKernelGGL(k_zpermute_b, dim3((total + 255) / 256), dim3(256), 0, st, k0p, kp, k0, k, Z, ldz, out);
    return hipGetLastError();
}

hipError_t launch_zchunk_prod(int nchunk, int k0, int k, int kp, int k0p, const dcplx* M, const dcplx* G, int64_t ldg,
                              int64_t gstride, dcplx* out, hipStream_t st) {
    const size_t shm = (size_t)(kp * k0p + kp * kp) * sizeof(dcplx);
    hipLaunchKernelGGL(k_zchunk_prod, dim3(nchunk), dim3(256), shm, st, k0, k, kp, k0p, M, G, ldg, gstride, out);
    return hipGetLastError();
}

}  // namespace tho
