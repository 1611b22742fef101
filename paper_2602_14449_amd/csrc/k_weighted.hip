// Row scaling for the two-stage method in a weighted inner product
// <x, y>_B = x^* diag(b) y (Algorithm 3 with a diagonal B): rows of V and A
// are multiplied by sqrt(b_i) before the Euclidean method, rows of its Q by
// 1 / sqrt(b_i) after it.
#include "tho_device.h"
#include "tho_internal.h"

namespace tho {

namespace {

// Y[i][j] = f(b_i) X[i][j] for i < n, j < w (w doubles per row), with
// f = sqrt (inv = 0) or 1 / sqrt (inv = 1).  One thread per element,
// consecutive threads along a row.
__global__ void k_row_scale(int64_t n, int w, const double* __restrict__ b, int inv, const double* X, int64_t ldx,
                            double* Y, int64_t ldy) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * w) return;
    const int64_t i = t / w;
    const int j = (int)(t % w);
    const double s = sqrt(b[i]);
    Y[i * ldy + j] = inv ? X[i * ldx + j] / s : X[i * ldx + j] * s;
}

}  // namespace

hipError_t launch_row_scale(int64_t n, int w, const double* b, int inv, const double* X, int64_t ldx, double* Y,
                            int64_t ldy, hipStream_t st) {
    if (n <= 0 || w <= 0) return hipSuccess;
    const int64_t nb = (n * w + 255) / 256;
    hipLaunchKernelGGL(k_row_scale, dim3((unsigned)nb), dim3(256), 0, st, n, w, b, inv, X, ldx, Y, ldy);
    return hipGetLastError();
}

}  // namespace tho
