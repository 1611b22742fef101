// Numerical-condition checks of tho_two_stage, reported through an int32
// info word at the start of the caller's workspace (read back by
// tho_get_info).  The word holds INT_MAX for "no condition"; each detected
// condition lowers it with atomicMin to its code, so the smallest code seen
// wins: 1 = non-finite value, 3 = ||V^* V - I||_F above the tolerance.
#include <climits>

#include "tho_device.h"
#include "tho_internal.h"

namespace tho {

namespace {

__global__ void k_info_reset(int* info) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *info = INT_MAX;
}

// Scan the outputs S (k0 x k) and R (k x k) for a value that is not finite
// (w = 1 real, 2 complex doubles per entry).  Every element of V and A is a
// factor in the reductions that produce them (V^* A, the column norms of the
// Householder QR and the products in between), and IEEE arithmetic keeps a
// NaN or an infinity non-finite through products and sums (0 * Inf = NaN),
// so a non-finite input always reaches S or R; so does an overflow inside
// the method.
__global__ void k_check_finite(int k0, int k, int w, const double* __restrict__ S, int64_t lds,
                               const double* __restrict__ R, int64_t ldr, int* info) {
    bool bad = false;
    const int ns = k0 * k * w, nr = k * k * w;
    for (int e = threadIdx.x; e < ns; e += blockDim.x) {
        const int i = e / (k * w), j = e % (k * w);
        bad |= !isfinite(S[(int64_t)i * lds * w + j]);
    }
    for (int e = threadIdx.x; e < nr; e += blockDim.x) {
        const int i = e / (k * w), j = e % (k * w);
        bad |= !isfinite(R[(int64_t)i * ldr * w + j]);
    }
    if (bad) atomicMin(info, 1);
}

// ||V^* V - I||_F from the Gram of V (real: G = V^T V; complex: the Gram of
// the real view [Re v_0, Im v_0, Re v_1, ...], from which
// (V^* V)_ij = G(2i,2j) + G(2i+1,2j+1) + i (G(2i,2j+1) - G(2i+1,2j))).  The
// Gram arrives as two column blocks, G0 = columns 0..63 (ld ld0) and
// G1 = columns 64.. (ld ld1).  One workgroup;
// the sum of squares is taken in a fixed order.  Sets code 3 above `tol`.
__global__ __launch_bounds__(256) void k_vorth_check(int k0, int cplx, const double* __restrict__ G0, int ld0,
                                                     const double* __restrict__ G1, int ld1, double tol, int* info) {
    __shared__ double red[256];
    auto g = [&](int i, int j) { return (j < 64) ? G0[i * ld0 + j] : G1[i * ld1 + (j - 64)]; };
    double s = 0.0;
    for (int e = threadIdx.x; e < k0 * k0; e += blockDim.x) {
        const int i = e / k0, j = e % k0;
        double re, im = 0.0;
        if (cplx) {
            re = g(2 * i, 2 * j) + g(2 * i + 1, 2 * j + 1);
            im = g(2 * i, 2 * j + 1) - g(2 * i + 1, 2 * j);
        } else {
            re = g(i, j);
        }
        if (i == j) re -= 1.0;
        s = fma(re, re, fma(im, im, s));
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double f = sqrt(red[0]);
        if (!(f <= tol)) atomicMin(info, 3);  // NaN counts as above
    }
}

}  // namespace

hipError_t launch_info_reset(int* info, hipStream_t st) {
    hipLaunchKernelGGL(k_info_reset, dim3(1), dim3(64), 0, st, info);
    return hipGetLastError();
}

hipError_t launch_check_finite(int k0, int k, int cplx, const double* S, int64_t lds, const double* R, int64_t ldr,
                               int* info, hipStream_t st) {
    if (k <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_check_finite, dim3(1), dim3(256), 0, st, k0, k, cplx ? 2 : 1, S, lds, R, ldr, info);
    return hipGetLastError();
}

hipError_t launch_vorth_check(int k0, int cplx, const double* G0, int ld0, const double* G1, int ld1, double tol,
                              int* info, hipStream_t st) {
    if (k0 <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_vorth_check, dim3(1), dim3(256), 0, st, k0, cplx, G0, ld0, G1, ld1, tol, info);
    return hipGetLastError();
}

}  // namespace tho
