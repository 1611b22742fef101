// Device-side helpers shared by the gfx950 kernels of libtho.
//
// FP64 MFMA (v_mfma_f64_16x16x4_f64) lane layouts on gfx950, as used
// throughout (l = lane in the 64-wide wavefront, v = accumulator element):
//   A operand (16x4, M x K):  lane l holds A[l % 16][l / 16]
//   B operand (4x16, K x N):  lane l holds B[l / 16][l % 16]
//   D/C (16x16):              lane l, element v holds D[l / 16 + 4 v][l % 16]
// A 16 x 16 block of a row-major matrix held "in D layout" therefore has its
// row index on (l / 16, v) and its column index on l % 16.  Such a block is
// directly usable as either operand of a product that contracts over its
// rows (take element v as the operand of the v-th K-step), which is how the
// kernels reduce over the n rows without moving data between lanes.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

typedef double d4 __attribute__((ext_vector_type(4)));

namespace tho {

constexpr int WAVE = 64;

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ d4 d4zero() {
    d4 z = {0.0, 0.0, 0.0, 0.0};
    return z;
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// Row (within a 16-row block) of accumulator element v of lane l.
__device__ __forceinline__ int drow(int l, int v) { return (l >> 4) + 4 * v; }

// Sum across the four 16-lane groups of a wavefront (lanes l, l^16, l^32,
// l^48 end up with the same value).
__device__ __forceinline__ double sum_groups(double x) {
    x += __shfl_xor(x, 16);
    x += __shfl_xor(x, 32);
    return x;
}

// Full wavefront sum.
__device__ __forceinline__ double sum_wave(double x) {
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

__device__ __forceinline__ double ldg(const double* p) { return __builtin_nontemporal_load(p); }

}  // namespace tho
