// Reduced-precision panel products for gfx950 (device side).
//
// Panel modes (tho_panel_t): 1 = FP32 hi + lo split, 2 = BF16.  Only the
// products of a row panel of V (n x k0) with a small k0 x k matrix use them
// (the update A + V Z and Q_ + V N); norms, reflectors and T stay FP64.
//
// FP32 hi + lo: an FP64 value x is split as hi = fl32(x), lo = fl32(x - hi);
// a product is hi*hi + hi*lo + lo*hi on v_mfma_f32_16x16x4_f32 (the lo*lo
// term is below FP32 resolution), accumulated in FP32 across the K loop of
// one tile and added to the FP64 accumulator at the end.
// BF16: operands rounded to bfloat16, v_mfma_f32_16x16x32_bf16, FP32
// accumulation, added to the FP64 accumulator.
//
// Lane layouts (gfx950): FP32-accumulating MFMAs return D[4*(l/16) + v][l%16],
// while the FP64 tile layout is D[l/16 + 4*v][l%16].  The A-operand lane that
// supplies MFMA row i therefore loads tile row pi(i) = i/4 + 4*(i%4), so that
// element (l, v) of the FP32 result is the FP64 tile element (l, v).
#pragma once

#include "tho_device.h"

namespace tho {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int PANEL_F64 = 0, PANEL_F32X2 = 1, PANEL_BF16 = 2;

__device__ __forceinline__ f4 mfma32(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfmabf(bf8 a, bf8 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 f4zero() {
    f4 z = {0.f, 0.f, 0.f, 0.f};
    return z;
}
__device__ __forceinline__ int lowp_row(int i) { return (i >> 2) + 4 * (i & 3); }

// Rows of the packed B operand: FP32 split uses K0P (K-steps of 4), BF16
// pads to a multiple of 32 (K-steps of 32).
__host__ __device__ constexpr int lowp_kpad(int panel, int k0p) {
    return panel == PANEL_BF16 ? (k0p < 32 ? 32 : k0p) : k0p;
}

// acc[rb][ct] (FP64 tile layout, rows wrow0 + 16 rb + ...) += V[rows, 0:k0] B,
// B packed by k_pack_b_lowp (K0P x 16 CT).  V rows at or beyond trows and
// columns at or beyond k0 read as zero.
template <int PANEL, int RB, int CT, int K0P>
__device__ __forceinline__ void vprod_lowp(d4 (&acc)[RB][CT], const double* __restrict__ Vt, int ldv, int wrow0,
                                           int trows, int k0, const void* __restrict__ Bp, int l) {
    const int g = l >> 4, cl = l & 15;
    if constexpr (PANEL == PANEL_F32X2) {
        constexpr int KS = K0P / 4;
        const float* Bh = (const float*)Bp;
        const float* Bl = Bh + KS * CT * 64;
#pragma unroll
        for (int rb = 0; rb < RB; rb++) {
            const int vr = wrow0 + 16 * rb + lowp_row(cl);
            const bool ok = vr < trows;
            const double* vp = Vt + vr * ldv + g * KS;
            f4 c[CT];
#pragma unroll
            for (int ct = 0; ct < CT; ct++) c[ct] = f4zero();
            constexpr int SC = (KS >= 8) ? 8 : KS;
#pragma unroll 2
            for (int s0 = 0; s0 < KS; s0 += SC) {
                float ah[SC], al[SC];
#pragma unroll
                for (int s = 0; s < SC; s++) {
                    const double a = (ok && g * KS + s0 + s < k0) ? vp[s0 + s] : 0.0;
                    ah[s] = (float)a;
                    al[s] = (float)(a - (double)ah[s]);
                }
#pragma unroll
                for (int s = 0; s < SC; s++)
#pragma unroll
                    for (int ct = 0; ct < CT; ct++) {
                        const float bh = Bh[((s0 + s) * CT + ct) * 64 + l];
                        const float bl = Bl[((s0 + s) * CT + ct) * 64 + l];
                        c[ct] = mfma32(ah[s], bh, c[ct]);
                        c[ct] = mfma32(ah[s], bl, c[ct]);
                        c[ct] = mfma32(al[s], bh, c[ct]);
                    }
            }
#pragma unroll
            for (int ct = 0; ct < CT; ct++)
#pragma unroll
                for (int v = 0; v < 4; v++) acc[rb][ct][v] += (double)c[ct][v];
        }
    } else {
        constexpr int KB = lowp_kpad(PANEL_BF16, K0P) / 4;  // columns per lane group
        constexpr int S8 = KB / 8;
        const bf8* B8 = (const bf8*)Bp;
#pragma unroll
        for (int rb = 0; rb < RB; rb++) {
            const int vr = wrow0 + 16 * rb + lowp_row(cl);
            const bool ok = vr < trows;
            const double* vp = Vt + vr * ldv + g * KB;
            f4 c[CT];
#pragma unroll
            for (int ct = 0; ct < CT; ct++) c[ct] = f4zero();
#pragma unroll
            for (int s = 0; s < S8; s++) {
                bf8 a;
#pragma unroll
                for (int e = 0; e < 8; e++) {
                    const int col = g * KB + 8 * s + e;
                    a[e] = (__bf16)(float)((ok && col < k0) ? vp[8 * s + e] : 0.0);
                }
#pragma unroll
                for (int ct = 0; ct < CT; ct++) c[ct] = mfmabf(a, B8[(s * CT + ct) * 64 + l], c[ct]);
            }
#pragma unroll
            for (int ct = 0; ct < CT; ct++)
#pragma unroll
                for (int v = 0; v < 4; v++) acc[rb][ct][v] += (double)c[ct][v];
        }
    }
}

}  // namespace tho
