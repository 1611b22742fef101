// Reduced-precision panel products (host-launched kernels): the split-n
// reduction C = V^T A with FP32 hi + lo or BF16 operands, and the packing of
// small FP64 matrices into the reduced-precision B-operand order used by the
// fused leaf / formation kernels (see tho_lowp.h for the arithmetic).
#include "tho_internal.h"
#include "tho_lowp.h"

namespace tho {

namespace {

// part[blk] = X[r0:r1]^T Y[r0:r1] (FP64 result, reduced-precision products).
// WM wave groups split the MT row tiles of the output, the 4/WM others split
// the rows; FP32 partial sums are folded into FP64 every FL K-steps.
// FP32 split: a K-step is 4 rows (lane group g reads row r + g).
// BF16:       a K-step is 32 rows (lane group g reads rows r + 8g + e).
template <int PANEL, int MT, int NT, int WM>
__global__ __launch_bounds__(256) void k_xty_lowp(int64_t nrows, const double* __restrict__ X, int64_t ldx, int p,
                                                 const double* __restrict__ Y, int64_t ldy, int q,
                                                 int64_t rows_per_blk, double* __restrict__ part) {
    constexpr int MTW = MT / WM;
    constexpr int WR = 4 / WM;
    constexpr int RED = (WR > 1) ? (WR - 1) * WM * MTW * NT * 64 : 1;
    constexpr int KR = (PANEL == PANEL_BF16) ? 32 : 4;  // rows per K-step
    constexpr int FL = (PANEL == PANEL_BF16) ? 2 : 8;   // K-steps per FP32 partial
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
    int colx[MTW], coly[NT];
#pragma unroll
    for (int i = 0; i < MTW; i++) colx[i] = 16 * (wm * MTW + i) + cl;
#pragma unroll
    for (int j = 0; j < NT; j++) coly[j] = 16 * j + cl;

    for (int64_t rb = r0 + (int64_t)wr * KR * FL; rb < r1; rb += (int64_t)WR * KR * FL) {
        f4 c[MTW][NT];
#pragma unroll
        for (int i = 0; i < MTW; i++)
#pragma unroll
            for (int j = 0; j < NT; j++) c[i][j] = f4zero();
#pragma unroll
        for (int u = 0; u < FL; u++) {
            if constexpr (PANEL == PANEL_F32X2) {
                const int64_t row = rb + 4 * u + g;
                const bool ok = row < r1;
                float xh[MTW], xl[MTW], yh[NT], yl[NT];
#pragma unroll
                for (int i = 0; i < MTW; i++) {
                    const double a = (ok && colx[i] < p) ? X[row * ldx + colx[i]] : 0.0;
                    xh[i] = (float)a;
                    xl[i] = (float)(a - (double)xh[i]);
                }
#pragma unroll
                for (int j = 0; j < NT; j++) {
                    const double b = (ok && coly[j] < q) ? Y[row * ldy + coly[j]] : 0.0;
                    yh[j] = (float)b;
                    yl[j] = (float)(b - (double)yh[j]);
                }
#pragma unroll
                for (int i = 0; i < MTW; i++)
#pragma unroll
                    for (int j = 0; j < NT; j++) {
                        c[i][j] = mfma32(xh[i], yh[j], c[i][j]);
                        c[i][j] = mfma32(xh[i], yl[j], c[i][j]);
                        c[i][j] = mfma32(xl[i], yh[j], c[i][j]);
                    }
            } else {
                const int64_t rowb = rb + 32 * u + 8 * g;
                bf8 xa[MTW], yb[NT];
#pragma unroll
                for (int e = 0; e < 8; e++) {
                    const int64_t row = rowb + e;
                    const bool ok = row < r1;
#pragma unroll
                    for (int i = 0; i < MTW; i++)
                        xa[i][e] = (__bf16)(float)((ok && colx[i] < p) ? X[row * ldx + colx[i]] : 0.0);
#pragma unroll
                    for (int j = 0; j < NT; j++)
                        yb[j][e] = (__bf16)(float)((ok && coly[j] < q) ? Y[row * ldy + coly[j]] : 0.0);
                }
#pragma unroll
                for (int i = 0; i < MTW; i++)
#pragma unroll
                    for (int j = 0; j < NT; j++) c[i][j] = mfmabf(xa[i], yb[j], c[i][j]);
            }
        }
#pragma unroll
        for (int i = 0; i < MTW; i++)
#pragma unroll
            for (int j = 0; j < NT; j++)
#pragma unroll
                for (int v = 0; v < 4; v++) acc[i][j][v] += (double)c[i][j][v];
    }
    // fold the WR row groups through LDS (fixed order)
    if (WR > 1) {
        if (wr > 0) {
#pragma unroll
            for (int i = 0; i < MTW; i++)
#pragma unroll
                for (int j = 0; j < NT; j++) red[(((wr - 1) * WM + wm) * MTW * NT + i * NT + j) * 64 + l] = acc[i][j];
        }
        __syncthreads();
        if (wr == 0) {
            for (int o = 1; o < WR; o++)
#pragma unroll
                for (int i = 0; i < MTW; i++)
#pragma unroll
                    for (int j = 0; j < NT; j++) acc[i][j] += red[(((o - 1) * WM + wm) * MTW * NT + i * NT + j) * 64 + l];
        }
    }
    if (wr == 0) {
        double* out = part + (int64_t)blockIdx.x * (16 * MT) * (16 * NT);
        // FP32-accumulator layout: element (l, v) is output row 4 * (l / 16) + v
#pragma unroll
        for (int i = 0; i < MTW; i++)
#pragma unroll
            for (int j = 0; j < NT; j++)
#pragma unroll
                for (int v = 0; v < 4; v++) {
                    const int row = 16 * (wm * MTW + i) + 4 * g + v;
                    out[row * (16 * NT) + 16 * j + cl] = acc[i][j][v];
                }
    }
}

// Reduced-precision B operand of vprod_lowp from a dense K0P x KP FP64
// matrix (ld KP, rows >= K0P read as zero).
//   FP32 split: hi[e], lo[e] for e = (s * CT + ct) * 64 + l, holding
//               B[(l/16) * (K0P/4) + s][16 ct + l%16]
//   BF16:       8 values per e = (s * CT + ct) * 64 + l, value j holding
//               B[(l/16) * (kpad/4) + 8 s + j][16 ct + l%16]
__global__ void k_pack_b_lowp(int panel, int K0P, int KP, const double* __restrict__ src, void* __restrict__ dst) {
    const int CT = KP / 16;
    if (panel == PANEL_F32X2) {
        const int KS = K0P / 4, n = KS * CT * 64;
        float* hi = (float*)dst;
        float* lo = hi + n;
        for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
            const int l = e & 63, sc = e >> 6, s = sc / CT, ct = sc % CT;
            const double b = src[((l >> 4) * KS + s) * KP + 16 * ct + (l & 15)];
            const float h = (float)b;
            hi[e] = h;
            lo[e] = (float)(b - (double)h);
        }
    } else {
        const int KB = lowp_kpad(PANEL_BF16, K0P) / 4, S8 = KB / 8, n = S8 * CT * 64;
        bf8* out = (bf8*)dst;
        for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
            const int l = e & 63, sc = e >> 6, s = sc / CT, ct = sc % CT;
            bf8 v;
            for (int j = 0; j < 8; j++) {
                const int r = (l >> 4) * KB + 8 * s + j;
                v[j] = (__bf16)(float)(r < K0P ? src[r * KP + 16 * ct + (l & 15)] : 0.0);
            }
            out[e] = v;
        }
    }
}

}  // namespace

size_t lowp_pack_bytes(int panel, int K0P, int KP) {
    if (panel == PANEL_F32X2) return (size_t)2 * K0P * KP * sizeof(float);
    return (size_t)lowp_kpad(PANEL_BF16, K0P) * KP * 2;
}

hipError_t launch_pack_b_lowp(int panel, int K0P, int KP, const double* src, void* dst, hipStream_t st) {
    hipLaunchKernelGGL(k_pack_b_lowp, dim3((K0P * KP + 255) / 256), dim3(256), 0, st, panel, K0P, KP, src, dst);
    return hipGetLastError();
}

#define XTYL_CASE(MT, NT, WM)                                                                              \
    if (mt == MT && nt == NT) {                                                                            \
        if (panel == PANEL_F32X2)                                                                          \
            hipLaunchKernelGGL((k_xty_lowp<PANEL_F32X2, MT, NT, WM>), dim3(nblk), dim3(256), 0, st, nrows, X, \
                               ldx, p, Y, ldy, q, rows_per_blk, part);                                     \
        else                                                                                               \
            hipLaunchKernelGGL((k_xty_lowp<PANEL_BF16, MT, NT, WM>), dim3(nblk), dim3(256), 0, st, nrows, X, \
                               ldx, p, Y, ldy, q, rows_per_blk, part);                                     \
        return hipGetLastError();                                                                          \
    }

hipError_t launch_xty_lowp(int panel, int mt, int nt, int64_t nrows, const double* X, int64_t ldx, int p,
                           const double* Y, int64_t ldy, int q, int nblk, int64_t rows_per_blk, double* part,
                           hipStream_t st) {
    if (panel != PANEL_F32X2 && panel != PANEL_BF16) return hipErrorInvalidValue;
    XTYL_CASE(1, 1, 1)
    XTYL_CASE(1, 2, 1)
    XTYL_CASE(1, 4, 1)
    XTYL_CASE(2, 1, 2)
    XTYL_CASE(2, 2, 2)
    XTYL_CASE(2, 4, 2)
    XTYL_CASE(4, 1, 4)
    XTYL_CASE(4, 2, 4)
    XTYL_CASE(4, 4, 4)
    XTYL_CASE(8, 1, 4)
    XTYL_CASE(8, 2, 4)
    XTYL_CASE(8, 4, 4)
    return hipErrorInvalidValue;
}

}  // namespace tho
