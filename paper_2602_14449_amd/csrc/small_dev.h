// Device routines shared by the single-problem and the batched kernels:
// the QR of the square top block of V (second choice of P, §3.2).
#pragma once

#include "tho_device.h"

namespace tho {

// Householder QR of the square top block V_top (n x n, n <= 128) with
// nonnegative diag(R) (the second choice of P, §3.2), entirely in LDS, then
//   P = -Q1  and  T = I + R1^T  (lower triangular; the form of Appendix B.2)
// written to P (ld n) and T (ld n).  Reflectors use the same convention as
// the rest of the library (beta = -sign(alpha) * norm, tau = 0 for a zero
// subcolumn); Q is formed in place from the reflectors (backward
// accumulation), then columns of Q / rows of R are scaled by sign(R_jj).
// Any block size that is a multiple of 128 (n > 64) or 64 (n <= 64) works;
// the columns are spread over CW lanes and the rows over blockDim / CW
// groups.  LDS: qr_top_lds(n) doubles at sm.
__host__ __device__ constexpr int qr_top_lds(int n) { return n * (n + 1) + 16 * n + 4 * n + 16; }

__device__ inline void qr_top_body(int n, const double* __restrict__ Vt, int64_t ldv, double* __restrict__ P,
                                   double* __restrict__ T, double* sm) {
    const int ld = n + 1;
    const int CW = (n > 64) ? 128 : 64;
    const int RG = (int)blockDim.x / CW;
    double* M = sm;                 // n x ld
    double* part = M + n * ld;      // RG (<= 16) x n partial dots
    double* wv = part + 16 * n;     // n: w_c of the current reflector
    double* taus = wv + n;          // n
    double* sgn = taus + n;         // n: sign of R_jj
    double* ub = sgn + n;           // n: the reflector being applied in the formation
    double* red = ub + n;           // 16 scalars
    const int tid = threadIdx.x;
    const int c = tid % CW, rg = tid / CW;  // column, row group
    for (int e = tid; e < n * n; e += blockDim.x) M[(e / n) * ld + (e % n)] = Vt[(int64_t)(e / n) * ldv + (e % n)];
    __syncthreads();
    // Two workgroup barriers per column.  Thread (c, rg) forms the partial
    // dot d_c = sum over its rows i > j of x_ij x_ic for every c >= j (c = j
    // gives sigma^2); after the barrier every thread builds the reflector
    // from sigma^2 and alpha = M[j][j] itself, and the threads of column c > j
    // apply it: w_c = M[j][c] + s d_c with u = [1; s x_sub], s = 1 / (alpha -
    // beta).  Column j is scaled after the second barrier; no later step of
    // the factorization reads it.
    for (int j = 0; j < n; j++) {
        if (c < n && c >= j) {
            double s = 0.0;
            for (int i = j + 1 + rg; i < n; i += RG) s += M[i * ld + j] * M[i * ld + c];
            part[rg * n + c] = s;
        }
        __syncthreads();
        double sig2 = 0.0;
        for (int r = 0; r < RG; r++) sig2 += part[r * n + j];
        const double alpha = M[j * ld + j];
        double beta = alpha, tau = 0.0, scale = 0.0;
        if (sig2 != 0.0) {
            const double nrm = sqrt(alpha * alpha + sig2);
            beta = (alpha < 0.0) ? nrm : -nrm;
            tau = (beta - alpha) / beta;
            scale = 1.0 / (alpha - beta);
        }
        // (every thread of column c reads the pivot-row entry M[j][c]; the
        // updated entry is stored after the barrier)
        double rowj = 0.0;
        if (c < n && c > j) {
            double d = 0.0;
            for (int r = 0; r < RG; r++) d += part[r * n + c];
            rowj = M[j * ld + c];
            const double tw = tau * (rowj + scale * d);
            const double tws = tw * scale;
            rowj -= tw;
            for (int i = j + 1 + rg; i < n; i += RG) M[i * ld + c] -= tws * M[i * ld + j];
        }
        __syncthreads();
        if (c < n && c > j && rg == 0) M[j * ld + c] = rowj;
        if (tid > j && tid < n) M[tid * ld + j] *= scale;
        if (tid == 0) {
            taus[j] = tau;
            M[j * ld + j] = beta;
        }
    }
    __syncthreads();
    // R1 diagonal signs and T = I + D R1^T (rows of R scaled by d)
    for (int e = tid; e < n * n; e += blockDim.x) {
        const int i = e / n, jj = e % n;  // T[i][jj] = delta + d_jj R[jj][i] for jj <= i
        double v = (i == jj) ? 1.0 : 0.0;
        if (jj <= i) {
            const double d = (M[jj * ld + jj] < 0.0) ? -1.0 : 1.0;
            v += d * M[jj * ld + i];
        }
        T[(int64_t)i * n + jj] = v;
    }
    // keep the diagonal signs before Q overwrites M
    if (tid < n) sgn[tid] = (M[tid * ld + tid] < 0.0) ? -1.0 : 1.0;
    __syncthreads();
    // form Q in place (backward accumulation of the reflectors), two
    // barriers per column: the dots copy the reflector u_j into ub, so that
    // the update reads it there while column j is overwritten by its formed
    // value H_j e_j in the same phase.  Row j of an already formed column
    // c > j is zero, so its update is -tau w_c and needs no read.
    for (int j = n - 1; j >= 0; j--) {
        const double tau = taus[j];
        if (j < n - 1) {
            if (c < n && c > j) {
                double s = 0.0;
                for (int i = j + 1 + rg; i < n; i += RG) s += M[i * ld + j] * M[i * ld + c];
                part[rg * n + c] = s;
            }
            for (int i = j + 1 + tid; i < n; i += blockDim.x) ub[i] = M[i * ld + j];
            __syncthreads();
            if (c < n && c > j) {
                double wc = 0.0;
                for (int r = 0; r < RG; r++) wc += part[r * n + c];
                const double tw = tau * wc;
                for (int i = j + 1 + rg; i < n; i += RG) M[i * ld + c] -= tw * ub[i];
                if (rg == 0) M[j * ld + c] = -tw;
            }
        }
        if (tid < n) {
            if (tid > j) M[tid * ld + j] = -tau * ub[tid];
            else if (tid == j) M[j * ld + j] = 1.0 - tau;
            else M[tid * ld + j] = 0.0;
        }
        __syncthreads();
    }
    // P = -Q D
    for (int e = tid; e < n * n; e += blockDim.x) {
        const int i = e / n, jj = e % n;
        P[(int64_t)i * n + jj] = -M[i * ld + jj] * sgn[jj];
    }
}

}  // namespace tho
