// Row-streaming panel products for gfx950:
//
//   Out[r, 0:q] = X[r, 0:q] + sum_t Y_t[r, 0:p_t] B_t          (r < nrows)
//
// with every B_t small (p_t x q) and pre-packed in FP64 MFMA B-operand order
// (k_pack_b).  This is the shape of every n-row update outside the fused
// leaf/formation kernels: the projections X - V C of block Gram-Schmidt, the
// re-formation of intermediates and the streaming terms of the adjoint
// (rows of V, A, Q and their adjoints times k0 x k or k x k matrices).
//
// Each wavefront owns RB 16-row blocks (RB = 4 up to 64 output columns,
// 2 for 128) and keeps the output block in MFMA accumulator layout, so X is
// read and Out written by the same lane (Out may alias X).  The contraction
// index of term t is split as rows_kidx(s, lane / 16): each batch of four
// K-steps reads one whole 128-byte line of every row it touches, the four
// lane groups side by side.
#include "tho_device.h"
#include "tho_internal.h"

namespace tho {

namespace {

template <int CT, int RB>
__global__ __launch_bounds__(256, 2) void k_rows_gemm(RowsGemm g) {
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6, gq = l >> 4, cl = l & 15;
    const int64_t wr0 = (int64_t)blockIdx.x * (4 * 16 * RB) + (int64_t)w * 16 * RB;
    const int64_t nrows = g.nrows;
    if (wr0 >= nrows) return;  // whole wavefront past the end (no barriers below)
    d4 acc[RB][CT];
#pragma unroll
    for (int rb = 0; rb < RB; rb++)
#pragma unroll
        for (int ct = 0; ct < CT; ct++)
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int64_t row = wr0 + 16 * rb + drow(l, v);
                const int col = 16 * ct + cl;
                acc[rb][ct][v] = (g.X && row < nrows && col < g.q) ? g.X[row * g.ldx + col] : 0.0;
            }
    for (int t = 0; t < g.nterm; t++) {
        const double* __restrict__ Y = g.t[t].Y;
        const double* __restrict__ B = g.t[t].B;
        const int64_t ldy = g.t[t].ldy;
        const int p = g.t[t].p, KS = g.t[t].kpad / 4;
        for (int s0 = 0; s0 < KS; s0 += 4) {
            double a[RB][4], b[4][CT];
#pragma unroll
            for (int rb = 0; rb < RB; rb++) {
                const int64_t row = wr0 + 16 * rb + cl;
#pragma unroll
                for (int s = 0; s < 4; s++) {
                    const int c = rows_kidx(s0 + s, gq);
                    a[rb][s] = (row < nrows && c < p) ? Y[row * ldy + c] : 0.0;
                }
            }
#pragma unroll
            for (int s = 0; s < 4; s++)
#pragma unroll
                for (int ct = 0; ct < CT; ct++) b[s][ct] = B[((s0 + s) * CT + ct) * 64 + l];
#pragma unroll
            for (int s = 0; s < 4; s++)
#pragma unroll
                for (int rb = 0; rb < RB; rb++)
#pragma unroll
                    for (int ct = 0; ct < CT; ct++) acc[rb][ct] = mfma(a[rb][s], b[s][ct], acc[rb][ct]);
        }
    }
#pragma unroll
    for (int rb = 0; rb < RB; rb++)
#pragma unroll
        for (int ct = 0; ct < CT; ct++)
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int64_t row = wr0 + 16 * rb + drow(l, v);
                const int col = 16 * ct + cl;
                if (row < nrows && col < g.q) g.Out[row * g.ldo + col] = acc[rb][ct][v];
            }
}

// dst (kpad x qp, B-operand order) = scale * op(src) zero-padded, where
// op(src)(i, j) = src[i*lds + j] (trans == 0) or src[j*lds + i] (trans == 1)
// for i < p, j < q.  Element e of dst: lane l = e % 64, K-step s and column
// tile ct from e / 64, holding B[rows_kidx(s, l/16)][16 ct + l%16].
__global__ void k_pack_b(int p, int q, const double* __restrict__ src, int64_t lds, int trans, double scale,
                         int kpad, int qp, double* __restrict__ dst) {
    const int n = kpad * qp, CT = qp / 16;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
        const int l = e & 63, sc = e >> 6, s = sc / CT, ct = sc % CT;
        const int i = rows_kidx(s, l >> 4), j = 16 * ct + (l & 15);
        double v = 0.0;
        if (i < p && j < q) v = scale * (trans ? src[(int64_t)j * lds + i] : src[(int64_t)i * lds + j]);
        dst[e] = v;
    }
}

}  // namespace

int rows_gemm_qp(int q) { return q <= 16 ? 16 : (q <= 32 ? 32 : (q <= 64 ? 64 : 128)); }

hipError_t launch_rows_gemm(const RowsGemm& g, hipStream_t st) {
    if (g.nrows <= 0 || g.q <= 0) return hipSuccess;
    if (g.q > 128 || g.nterm < 0 || g.nterm > RowsGemm::MAXT) return hipErrorInvalidValue;
    for (int t = 0; t < g.nterm; t++)
        if (g.t[t].kpad % 16 != 0 || g.t[t].p > g.t[t].kpad) return hipErrorInvalidValue;
    const int qp = rows_gemm_qp(g.q);
    if (qp == 128) {
        const unsigned nb = (unsigned)((g.nrows + 127) / 128);
        hipLaunchKernelGGL((k_rows_gemm<8, 2>), dim3(nb), dim3(256), 0, st, g);
    } else {
        const unsigned nb = (unsigned)((g.nrows + 255) / 256);
        if (qp == 16) hipLaunchKernelGGL((k_rows_gemm<1, 4>), dim3(nb), dim3(256), 0, st, g);
        else if (qp == 32) hipLaunchKernelGGL((k_rows_gemm<2, 4>), dim3(nb), dim3(256), 0, st, g);
        else hipLaunchKernelGGL((k_rows_gemm<4, 4>), dim3(nb), dim3(256), 0, st, g);
    }
    return hipGetLastError();
}

hipError_t launch_pack_b(int p, int q, const double* src, int64_t lds, int trans, double scale, int kpad, int qp,
                         double* dst, hipStream_t st) {
    const int n = kpad * qp;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pack_b, dim3((n + 255) / 256), dim3(256), 0, st, p, q, src, lds, trans, scale, kpad, qp,
                       dst);
    return hipGetLastError();
}

}  // namespace tho
