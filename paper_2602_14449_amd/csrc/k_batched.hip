// Batched two-stage orthogonalization: many independent (V, A) problems of
// uneven sizes in one persistent launch.
//
// Every workgroup loops: it takes the next problem from a device counter
// (problems are ordered longest first on the host) and runs all of
// Algorithm 1 (second choice of P) for that problem by itself:
//   QR of V_top -> P, T;  C = V^T A over all rows;  Z = T^{-T}(P^T A_top - C);
//   A1_top, S;  Householder QR of A_low + V_low Z as one chunk of tiles
//   (the same device code as the single-problem leaf, accumulating
//   N = V_low^T Q_loc);  R with nonnegative diagonal;  N = -T^{-1} N_c D;
//   Q_top;  formation of Q_low = Q_ + V_low N (the same formation code).
// A problem is one TSQR chunk, so there is no reduction tree and no
// grid-wide synchronization; the only shared state is the work counter,
// which every workgroup reads until the problems run out.
#include "small_dev.h"
#include "tsqr_dev.h"

namespace tho {

namespace {

constexpr int BW = 256;  // threads per workgroup (LEAF_WAVES wavefronts)

// Cs (16 MT x 16 NT, ld 16 NT + 1, LDS) = X^T Y over rows [0, n).  Wavefront
// w takes 16-row blocks w, w + 4, ...; the four partial sums are added in
// wavefront order (deterministic).
template <int MT, int NT>
__device__ void wg_xty(int64_t n, const double* __restrict__ X, int64_t ldx, int p, const double* __restrict__ Y,
                       int64_t ldy, int q, double* Cs) {
    constexpr int LDC = 16 * NT + 1;
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6, g = l >> 4, cl = l & 15;
    d4 acc[MT][NT];
#pragma unroll
    for (int i = 0; i < MT; i++)
#pragma unroll
        for (int j = 0; j < NT; j++) acc[i][j] = d4zero();
    for (int64_t rb = 16 * w; rb < n; rb += 64) {
        double xa[4][MT], yb[4][NT];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int64_t row = rb + 4 * u + g;
            const bool ok = row < n;
#pragma unroll
            for (int i = 0; i < MT; i++) xa[u][i] = (ok && 16 * i + cl < p) ? X[row * ldx + 16 * i + cl] : 0.0;
#pragma unroll
            for (int j = 0; j < NT; j++) yb[u][j] = (ok && 16 * j + cl < q) ? Y[row * ldy + 16 * j + cl] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; u++)
#pragma unroll
            for (int i = 0; i < MT; i++)
#pragma unroll
                for (int j = 0; j < NT; j++) acc[i][j] = mfma(xa[u][i], yb[u][j], acc[i][j]);
    }
    for (int o = 0; o < LEAF_WAVES; o++) {
        if (w == o) {
#pragma unroll
            for (int i = 0; i < MT; i++)
#pragma unroll
                for (int j = 0; j < NT; j++)
#pragma unroll
                    for (int v = 0; v < 4; v++) {
                        double* d = &Cs[(16 * i + drow(l, v)) * LDC + 16 * j + cl];
                        *d = (o == 0 ? 0.0 : *d) + acc[i][j][v];
                    }
        }
        __syncthreads();
    }
}

__device__ __forceinline__ double sgn1(double x) { return x < 0.0 ? -1.0 : 1.0; }

template <int KP, int K0P, int RBO>
__device__ __forceinline__ void run_instance(const BatchedInst& I, const TsqrLevel& L) {
    extern __shared__ double sm[];
    constexpr int LDC = KP + 1, CT = KP / 16;
    const int tid = threadIdx.x;
    const int k0 = I.k0, k = I.k;
    if constexpr (K0P > 0) {
        // second choice of P: V_top = Q1 R1, P = -Q1, T = I + R1^T
        qr_top_body(k0, I.V, I.ldv, I.Pm, I.Tm, sm);
        __syncthreads();
        double* Cs = sm;              // C = V^T A, later A1_top
        double* Zs = Cs + K0P * LDC;  // Y, then Z
        wg_xty<K0P / 16, KP / 16>(I.n, I.V, I.ldv, k0, I.A, I.lda, k, Cs);
        const double* Pm = I.Pm;
        const double* Tm = I.Tm;
        for (int e = tid; e < K0P * KP; e += BW) {
            const int i = e / KP, j = e % KP;
            double s = 0.0;
            if (i < k0 && j < k) {
                for (int p = 0; p < k0; p++) s = fma(Pm[p * k0 + i], I.A[p * I.lda + j], s);
                s -= Cs[i * LDC + j];
            }
            Zs[i * LDC + j] = s;
        }
        __syncthreads();
        // Z = T^{-T} Y (T^T upper): one column per thread
        if (tid < k) {
            for (int i = k0 - 1; i >= 0; i--) {
                double s = Zs[i * LDC + tid];
                for (int p = i + 1; p < k0; p++) s -= Tm[p * k0 + i] * Zs[p * LDC + tid];
                Zs[i * LDC + tid] = s / Tm[i * k0 + i];
            }
        }
        __syncthreads();
        for (int e = tid; e < K0P * KP; e += BW) {
            const int ln = e & 63, sc = e >> 6, s = sc / CT, ct = sc % CT;
            I.Zperm[e] = Zs[rows_kidx(s, ln >> 4) * LDC + 16 * ct + (ln & 15)];
        }
        // A1_top = A_top - (P - V_top) Z
        for (int e = tid; e < k0 * k; e += BW) {
            const int i = e / k, j = e % k;
            double s = I.A[i * I.lda + j];
            for (int p = 0; p < k0; p++) s -= (Pm[i * k0 + p] - I.V[i * I.ldv + p]) * Zs[p * LDC + j];
            Cs[i * LDC + j] = s;
        }
        __syncthreads();
        // S = P^T A1_top
        for (int e = tid; e < k0 * k; e += BW) {
            const int i = e / k, j = e % k;
            double s = 0.0;
            for (int p = 0; p < k0; p++) s = fma(Pm[p * k0 + i], Cs[p * LDC + j], s);
            I.S[i * I.lds + j] = s;
        }
        __syncthreads();
    }
    // Householder QR of A_low + V_low Z (one chunk); R -> Rtop, N_c^T -> Nc
    leaf_chunk<KP, K0P, 0, RBO>(L, 0);
    __syncthreads();
    const double* Rt = I.Rtop;
    for (int e = tid; e < k * k; e += BW) {
        const int i = e / k, j = e % k;
        I.R[i * I.ldr + j] = (j >= i) ? sgn1(Rt[i * KP + i]) * Rt[i * KP + j] : 0.0;
    }
    for (int e = tid; e < KP * KP; e += BW) {
        const int i = e / KP, j = e % KP;
        I.G0[e] = (i == j && i < k) ? sgn1(Rt[i * KP + i]) : 0.0;
    }
    if constexpr (K0P > 0) {
        const double* Pm = I.Pm;
        const double* Tm = I.Tm;
        double* Ns = sm;
        // G = W^T [0; Q_] = -N_c D ;  N = T^{-1} G
        for (int e = tid; e < K0P * KP; e += BW) {
            const int i = e / KP, j = e % KP;
            Ns[i * LDC + j] = (i < k0 && j < k) ? -I.Nc[j * K0P + i] * sgn1(Rt[j * KP + j]) : 0.0;
        }
        __syncthreads();
        if (tid < k) {
            for (int i = 0; i < k0; i++) {
                double s = Ns[i * LDC + tid];
                for (int p = 0; p < i; p++) s -= Tm[i * k0 + p] * Ns[p * LDC + tid];
                Ns[i * LDC + tid] = s / Tm[i * k0 + i];
            }
        }
        __syncthreads();
        for (int e = tid; e < K0P * KP; e += BW) {
            const int ln = e & 63, sc = e >> 6, s = sc / CT, ct = sc % CT;
            I.Nperm[e] = Ns[rows_kidx(s, ln >> 4) * LDC + 16 * ct + (ln & 15)];
        }
        // Q_top = -(P - V_top) N
        for (int e = tid; e < k0 * k; e += BW) {
            const int i = e / k, j = e % k;
            double s = 0.0;
            for (int p = 0; p < k0; p++) s -= (Pm[i * k0 + p] - I.V[i * I.ldv + p]) * Ns[p * LDC + j];
            I.Q[i * I.ldq + j] = s;
        }
    }
    __syncthreads();
    // rows of Q below k0 (overwrite the Householder vectors)
    form_chunk<KP, K0P, 0, RBO>(L, 0);
    __syncthreads();
}

// One kernel per (column class, V width class): a single inlined instance
// routine keeps the register allocation of the single-problem kernels.
template <int KP, int K0P, int RBO>
__global__ __launch_bounds__(BW, 2) void k_batched(const BatchedInst* __restrict__ insts,
                                                  const TsqrLevel* __restrict__ levels, const int* __restrict__ order,
                                                  int count, int* counter) {
    __shared__ int s_next;
    for (;;) {
        if (threadIdx.x == 0) s_next = atomicAdd(counter, 1);
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(s_next);
        __syncthreads();
        if (it >= count) break;  // uniform: every wavefront leaves together
        const int i = __builtin_amdgcn_readfirstlane(order[it]);
        const BatchedInst& I = insts[i];
        const TsqrLevel& L = levels[i];
        run_instance<KP, K0P, RBO>(I, L);
    }
}

__global__ void k_zero_ints(int* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

template <int KP, int RBO>
constexpr size_t batched_lds() {
    constexpr size_t pre = (size_t)2 * 64 * (KP + 1);
    constexpr size_t qr = (size_t)qr_top_lds(64);
    constexpr size_t leaf = LeafLds<KP, RBO>::total;
    constexpr size_t form = FormLds<KP>::total;
    return (pre > qr ? (pre > leaf ? (pre > form ? pre : form) : (leaf > form ? leaf : form))
                     : (qr > leaf ? (qr > form ? qr : form) : (leaf > form ? leaf : form))) *
           sizeof(double);
}

template <int KP, int K0P, int RBO>
hipError_t batched_t(const BatchedInst* insts, const TsqrLevel* levels, const int* order, int count, int* counter,
                     int grid, hipStream_t st) {
    constexpr size_t shm = batched_lds<KP, RBO>();
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void*)k_batched<KP, K0P, RBO>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL((k_batched<KP, K0P, RBO>), dim3(grid), dim3(BW), shm, st, insts, levels, order, count,
                       counter);
    return hipGetLastError();
}

template <int KP, int RBO>
hipError_t batched_k0(int k0p, const BatchedInst* insts, const TsqrLevel* levels, const int* order, int count,
                      int* counter, int grid, hipStream_t st) {
    switch (k0p) {
        case 0: return batched_t<KP, 0, RBO>(insts, levels, order, count, counter, grid, st);
        case 16: return batched_t<KP, 16, RBO>(insts, levels, order, count, counter, grid, st);
        case 32: return batched_t<KP, 32, RBO>(insts, levels, order, count, counter, grid, st);
        case 64: return batched_t<KP, 64, RBO>(insts, levels, order, count, counter, grid, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

int batched_tile_rows(int kp, int rbo) { return LEAF_WAVES * 16 * (rbo ? rbo : (kp >= 64 ? 2 : 4)); }

hipError_t launch_zero_ints(int* p, int n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_ints, dim3((n + 255) / 256), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

hipError_t launch_batched(int kp, int k0p, int rbo, const BatchedInst* insts, const TsqrLevel* levels,
                          const int* order, int count, int* counter, int grid, hipStream_t st) {
    switch (kp * 10 + rbo) {
        case 162: return batched_k0<16, 2>(k0p, insts, levels, order, count, counter, grid, st);
        case 164: return batched_k0<16, 4>(k0p, insts, levels, order, count, counter, grid, st);
        case 322: return batched_k0<32, 2>(k0p, insts, levels, order, count, counter, grid, st);
        case 324: return batched_k0<32, 4>(k0p, insts, levels, order, count, counter, grid, st);
        case 642: return batched_k0<64, 2>(k0p, insts, levels, order, count, counter, grid, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace tho
