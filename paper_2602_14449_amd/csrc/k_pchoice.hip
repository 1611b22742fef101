// The first and third choices of P (§3.2) for the k0 x k0 top block of V,
// each in one workgroup on the side stream (k0 <= 128):
//   first choice   modified LU (Algorithm 2): P diagonal, P - V_top = L U
//   third choice   polar decomposition V_top = Q2 M (one-sided Jacobi SVD,
//                  then a Householder QR of the rotated block), P = -Q2,
//                  T = I + M by Cholesky
// and the Cholesky factorization used by the third choice.
#include "small_dev.h"
#include "tho_internal.h"

namespace tho {

namespace {

// Modified LU of Z = V_top (n x n, n <= 128) in LDS, right-looking, one
// workgroup.  At step i the pivot sign is chosen from the updated Z_ii:
// P_ii = -sign(Z_ii) (sign(0) = +1), U_ii = P_ii - Z_ii, U_ij = -Z_ij,
// L_ji = -Z_ji / U_ii, and the trailing block is updated
// Z_jc += L_ji U_ic = Z_ji Z_ic / U_ii.  Outputs (ld n):
//   P   diag(P_ii)
//   F1  P L       (lower triangular, diagonal P_ii)
//   F2  U^T       (lower triangular, diagonal U_ii)
// so that T = (P - V_top)^T P = U^T L^T P is solved as
//   T^{-T} y = U^{-1} (P L)^{-1} y   and   T^{-1} y = (L^T P)^{-1} U^{-T} y.
__global__ __launch_bounds__(1024) void k_mlu_top(int n, const double* __restrict__ Vt, int64_t ldv,
                                                  double* __restrict__ P, double* __restrict__ F1,
                                                  double* __restrict__ F2) {
    extern __shared__ double sm[];
    const int ld = n + 1;
    double* M = sm;            // n x ld
    double* piv = M + n * ld;  // n: P_ii
    double* uii = piv + n;     // n: U_ii
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int e = tid; e < n * n; e += nt) M[(e / n) * ld + (e % n)] = Vt[(int64_t)(e / n) * ldv + (e % n)];
    __syncthreads();
    for (int i = 0; i < n; i++) {
        const double z = M[i * ld + i];
        const double p = (z >= 0.0) ? -1.0 : 1.0;
        const double u = p - z;  // |u| >= 1
        const double ru = 1.0 / u;
        if (tid == 0) { piv[i] = p; uii[i] = u; }
        const int m = n - 1 - i;  // trailing size
        for (int e = tid; e < m * m; e += nt) {
            const int j = i + 1 + e / m, c = i + 1 + e % m;
            M[j * ld + c] = fma(M[j * ld + i] * ru, M[i * ld + c], M[j * ld + c]);
        }
        __syncthreads();
    }
    for (int e = tid; e < n * n; e += nt) {
        const int r = e / n, c = e % n;
        double f1 = 0.0, f2 = 0.0;
        if (r == c) {
            f1 = piv[r];
            f2 = uii[r];
        } else if (r > c) {
            f1 = piv[r] * (-M[r * ld + c] / uii[c]);  // (P L)_rc = P_rr L_rc
            f2 = -M[c * ld + r];                    // (U^T)_rc = U_cr = -Z_cr
        }
        F1[e] = f1;
        F2[e] = f2;
        P[e] = (r == c) ? piv[r] : 0.0;
    }
}

// One-sided (Hestenes) Jacobi on the columns of V_top (n x n, n <= 128):
// B = V_top W with mutually orthogonal columns, W orthogonal (the product of
// the plane rotations).  Rounds of the round-robin ordering rotate n/2
// disjoint column pairs at once; 16 threads share a pair (rows split
// 16 ways).  A pair (p, q) is rotated when |b_p . b_q| > tol ||b_p|| ||b_q||,
// with t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)), zeta = (||b_q||^2 -
// ||b_p||^2) / (2 b_p . b_q), c = 1 / sqrt(1 + t^2), s = c t:
//   b_p <- c b_p - s b_q,  b_q <- s b_p + c b_q  (same on W).
// Sweeps stop after one without rotations (at most JAC_SWEEPS).  B lives
// in LDS, W in global memory (visible across the workgroup after each
// barrier).  Outputs B and W, ld n.
constexpr int JAC_SWEEPS = 40;

__global__ __launch_bounds__(1024) void k_jacobi_top(int n, const double* __restrict__ Vt, int64_t ldv,
                                                     double* __restrict__ Bout, double* __restrict__ W,
                                                     double* __restrict__ Wout) {
    extern __shared__ double sm[];
    const int np = n + (n & 1);  // even number of columns (a zero column pads odd n)
    const int ld = np + 1;
    double* B = sm;                     // n x ld
    int* flag = (int*)(B + n * ld);     // rotations in this sweep; then np ranks
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int e = tid; e < n * np; e += nt) {
        const int r = e / np, c = e % np;
        B[r * ld + c] = (c < n) ? Vt[(int64_t)r * ldv + c] : 0.0;
    }
    for (int e = tid; e < np * np; e += nt) W[e] = ((e / np) == (e % np)) ? 1.0 : 0.0;
    const double tol = 4.0 * sqrt((double)n) * 1.1102230246251565e-16;
    const int grp = tid >> 4, gl = tid & 15;  // pair slot, lane within the pair
    const int npairs = np / 2;
    for (int sweep = 0; sweep < JAC_SWEEPS; sweep++) {
        if (tid == 0) *flag = 0;
        __syncthreads();
        for (int rnd = 0; rnd < np - 1; rnd++) {
            if (grp < npairs) {
                // round-robin: position 0 fixed, positions 1..np-1 rotate
                auto player = [&](int pos) { return pos == 0 ? 0 : 1 + (pos - 1 + rnd) % (np - 1); };
                int p = player(grp), q = player(np - 1 - grp);
                if (p > q) { const int t = p; p = q; q = t; }
                double a = 0.0, b = 0.0, g = 0.0;
                for (int r = gl; r < n; r += 16) {
                    const double x = B[r * ld + p], y = B[r * ld + q];
                    a = fma(x, x, a);
                    b = fma(y, y, b);
                    g = fma(x, y, g);
                }
                // fixed-order sums over the 16 lanes, then lane 0's value in all
#pragma unroll
                for (int o = 8; o >= 1; o >>= 1) {
                    a += __shfl_xor(a, o, 16);
                    b += __shfl_xor(b, o, 16);
                    g += __shfl_xor(g, o, 16);
                }
                a = __shfl(a, 0, 16);
                b = __shfl(b, 0, 16);
                g = __shfl(g, 0, 16);
                if (g != 0.0 && fabs(g) > tol * sqrt(a) * sqrt(b)) {
                    const double zeta = (b - a) / (2.0 * g);
                    const double t = ((zeta >= 0.0) ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                    const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
                    for (int r = gl; r < n; r += 16) {
                        const double x = B[r * ld + p], y = B[r * ld + q];
                        B[r * ld + p] = c * x - s * y;
                        B[r * ld + q] = s * x + c * y;
                    }
                    for (int r = gl; r < np; r += 16) {
                        const double x = W[r * np + p], y = W[r * np + q];
                        W[r * np + p] = c * x - s * y;
                        W[r * np + q] = s * x + c * y;
                    }
                    if (gl == 0) *flag = 1;
                }
            }
            __syncthreads();
        }
        const int any = *flag;
        __syncthreads();
        if (!any) break;
    }
    // columns sorted by decreasing norm (B W^T is unchanged when B and W
    // are permuted alike): the Householder QR of B then meets any zero
    // columns last, where they leave R diagonal
    int* rank = flag + 2;                      // np entries (np is even)
    double* nrm = (double*)(flag + 2 + np);    // np squared column norms, 8-byte aligned
    for (int c = tid; c < np; c += nt) {
        double s = 0.0;
        for (int r = 0; r < n; r++) s = fma(B[r * ld + c], B[r * ld + c], s);
        nrm[c] = s;
    }
    __syncthreads();
    for (int c = tid; c < np; c += nt) {
        int rk = 0;
        for (int c2 = 0; c2 < np; c2++) rk += (nrm[c2] > nrm[c] || (nrm[c2] == nrm[c] && c2 < c)) ? 1 : 0;
        rank[c] = rk;
    }
    __syncthreads();
    for (int e = tid; e < n * np; e += nt) {
        const int r = e / np, c = e % np;
        if (rank[c] < n) Bout[r * n + rank[c]] = B[r * ld + c];
    }
    for (int e = tid; e < np * np; e += nt) {
        const int r = e / np, c = e % np;
        Wout[r * np + rank[c]] = W[r * np + c];
    }
}

// C = chol(I + (M + M^T) / 2), lower triangular, ld n (n <= 128), right-
// looking in LDS.  I + sym(M) is the T of the third choice (M the Hermitian
// polar factor, ||M||_2 <= 1), positive definite with kappa <= 2.
__global__ __launch_bounds__(1024) void k_chol_top(int n, const double* __restrict__ Min, int64_t ldm,
                                                   double* __restrict__ C) {
    extern __shared__ double sm[];
    const int ld = n + 1;
    double* A = sm;
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int e = tid; e < n * n; e += nt) {
        const int r = e / n, c = e % n;
        A[r * ld + c] = ((r == c) ? 1.0 : 0.0) + 0.5 * (Min[(int64_t)r * ldm + c] + Min[(int64_t)c * ldm + r]);
    }
    __syncthreads();
    for (int j = 0; j < n; j++) {
        const double d = sqrt(A[j * ld + j]);
        const double rd = 1.0 / d;
        __syncthreads();  // every thread has read A[j][j]
        if (tid == 0) A[j * ld + j] = d;
        for (int i = j + 1 + tid; i < n; i += nt) A[i * ld + j] *= rd;
        __syncthreads();
        const int m = n - 1 - j;
        for (int e = tid; e < m * m; e += nt) {
            const int i = j + 1 + e / m, c = j + 1 + e % m;
            if (c <= i) A[i * ld + c] = fma(-A[i * ld + j], A[c * ld + j], A[i * ld + c]);
        }
        __syncthreads();
    }
    for (int e = tid; e < n * n; e += nt) {
        const int r = e / n, c = e % n;
        C[e] = (c <= r) ? A[r * ld + c] : 0.0;
    }
}

hipError_t set_lds_limit(const void* k) {
    return hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

}  // namespace

size_t pchoice_ws_doubles(int n) { return 5 * (size_t)(n + 2) * (n + 2); }

hipError_t launch_mlu_top(int n, const double* Vt, int64_t ldv, double* P, double* F1, double* F2, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    static hipError_t attr = set_lds_limit((const void*)k_mlu_top);
    if (attr != hipSuccess) return attr;
    const size_t shm = ((size_t)n * (n + 1) + 2 * n) * sizeof(double);
    hipLaunchKernelGGL(k_mlu_top, dim3(1), dim3(1024), shm, st, n, Vt, ldv, P, F1, F2);
    return hipGetLastError();
}

// Third choice: P = -Q2 and C = chol(I + M), V_top = Q2 M.  After the Jacobi
// rotations B = V_top W has orthogonal columns; the Householder QR of B with
// nonnegative diagonal, B = Q_B R_B (R_B diagonal up to the Jacobi
// tolerance), gives V_top = Q_B R_B W^T, so Q2 = Q_B W^T and
// M = Q2^T V_top (symmetric up to that tolerance; symmetrized before the
// Cholesky factorization).  ws holds pchoice_ws_doubles(n) doubles.
hipError_t launch_polar_top(int n, const double* Vt, int64_t ldv, double* P, double* C, double* ws, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    static hipError_t attr1 = set_lds_limit((const void*)k_jacobi_top);
    static hipError_t attr2 = set_lds_limit((const void*)k_chol_top);
    if (attr1 != hipSuccess) return attr1;
    if (attr2 != hipSuccess) return attr2;
    const int np = n + (n & 1);
    double* B = ws;                               // n x n
    double* Wm = B + (size_t)(n + 1) * (n + 1);   // np x np
    double* PB = Wm + (size_t)(n + 1) * (n + 1);  // n x n: -Q_B
    double* TB = PB + (size_t)(n + 1) * (n + 1);  // n x n: scratch (I + R_B^T), then M
    double* W0 = TB + (size_t)(n + 1) * (n + 1);  // np x np: W before the sort
    const size_t shm1 = (size_t)n * (np + 1) * sizeof(double) + (size_t)(2 * np + 4) * sizeof(int) +
                        (size_t)np * sizeof(double);
    hipLaunchKernelGGL(k_jacobi_top, dim3(1), dim3(1024), shm1, st, n, Vt, ldv, B, W0, Wm);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((e = launch_qr_top(n, B, n, PB, TB, st)) != hipSuccess) return e;
    // P0 = -Q2 = (-Q_B) W^T  (W is np x np; its leading n x n block).  W is a
    // product of many rotations (tens of thousands at n = 128), orthogonal
    // only to about that many roundings; one Newton-Schulz step,
    // P = P0 (3 I - P0^T P0) / 2, brings P back to orthogonal at rounding
    // level (it moves P by the same small amount, and M below is formed
    // from the final P)
    double* P0 = W0;  // free after the Jacobi kernel
    if ((e = launch_small_gemm(n, n, n, 1.0, PB, n, 0, Wm, np, 1, 0.0, nullptr, 0, P0, n, st)) != hipSuccess) return e;
    if ((e = launch_small_gemm(n, n, n, 1.0, P0, n, 1, P0, n, 0, 0.0, nullptr, 0, TB, n, st)) != hipSuccess) return e;
    if ((e = launch_small_gemm(n, n, n, -0.5, P0, n, 0, TB, n, 0, 1.5, P0, n, P, n, st)) != hipSuccess) return e;
    // M = Q2^T V_top = -P^T V_top
    if ((e = launch_small_gemm(n, n, n, -1.0, P, n, 1, Vt, ldv, 0, 0.0, nullptr, 0, TB, n, st)) != hipSuccess)
        return e;
    const size_t shm2 = (size_t)n * (n + 1) * sizeof(double);
    hipLaunchKernelGGL(k_chol_top, dim3(1), dim3(1024), shm2, st, n, TB, (int64_t)n, C);
    return hipGetLastError();
}

}  // namespace tho
