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

// ---- cross-lane moves on VALU (no LDS crossbar)
__device__ __forceinline__ unsigned dlo(double x) { return (unsigned)__double_as_longlong(x); }
__device__ __forceinline__ unsigned dhi(double x) { return (unsigned)(__double_as_longlong(x) >> 32); }
__device__ __forceinline__ double dmake(unsigned lo, unsigned hi) {
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// v_permlane16_swap with both operands x: every lane receives the pair
// (value of its lane in the even 16-lane row, value in the odd row) of its
// 32-lane half.
struct dpair {
    double even, odd;
};
__device__ __forceinline__ dpair pair16(double x) {
    const auto lo = __builtin_amdgcn_permlane16_swap(dlo(x), dlo(x), false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap(dhi(x), dhi(x), false, false);
    return {dmake(lo[0], hi[0]), dmake(lo[1], hi[1])};
}
// v_permlane32_swap: (value in the lower 32-lane half, value in the upper half).
__device__ __forceinline__ dpair pair32(double x) {
    const auto lo = __builtin_amdgcn_permlane32_swap(dlo(x), dlo(x), false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(dhi(x), dhi(x), false, false);
    return {dmake(lo[0], hi[0]), dmake(lo[1], hi[1])};
}

// v_permlane16_swap / v_permlane32_swap on two different doubles (no
// copies): swap16 exchanges the odd 16-lane rows of a with the even rows of
// b; swap32 exchanges the upper 32-lane half of a with the lower half of b.
__device__ __forceinline__ void swap16(double& a, double& b) {
    const auto lo = __builtin_amdgcn_permlane16_swap(dlo(a), dlo(b), false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap(dhi(a), dhi(b), false, false);
    a = dmake(lo[0], hi[0]);
    b = dmake(lo[1], hi[1]);
}
__device__ __forceinline__ void swap32(double& a, double& b) {
    const auto lo = __builtin_amdgcn_permlane32_swap(dlo(a), dlo(b), false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(dhi(a), dhi(b), false, false);
    a = dmake(lo[0], hi[0]);
    b = dmake(lo[1], hi[1]);
}

// Column sums of CT per-lane partial values s[ct] (lane l holding a partial
// for column 16 ct + l % 16): returns, in lane l < 16 CT, the sum over the
// four 16-lane groups for column l.  Two values share every swap, so no
// lane moves are spent on copies (CT = 4: four permlane16 and two
// permlane32 swaps, three adds).
template <int CT>
__device__ __forceinline__ double col_sums(double (&s)[CT]) {
    if constexpr (CT == 4) {
        double a = s[0], b = s[1], c = s[2], d = s[3];
        swap16(a, b);  // a: rows (0+1 of s0, 0+1 of s1, 2+3 of s0, 2+3 of s1) after a + b
        swap16(c, d);
        double p = a + b, q = c + d;
        swap32(p, q);  // p + q: row r holds the total of s[r]
        return p + q;
    } else if constexpr (CT == 2) {
        double a = s[0], b = s[1];
        swap16(a, b);
        double p = a + b, q = p;
        swap32(p, q);  // rows 0 and 1 hold the totals of s[0] and s[1]
        return p + q;
    } else {
        const dpair e = pair16(s[0]);
        const dpair f = pair32(e.even + e.odd);
        return f.even + f.odd;
    }
}

// Sum across the four 16-lane groups of a wavefront (lanes l, l^16, l^32,
// l^48 end up with the same value, bitwise).
__device__ __forceinline__ double sum_groups(double x) {
    const dpair a = pair16(x);
    const dpair b = pair32(a.even + a.odd);
    return b.even + b.odd;
}

// Sum across the four lanes of a quad (DPP quad_perm).
__device__ __forceinline__ double sum_quad(double x) {
    const double y = dmake((unsigned)__builtin_amdgcn_mov_dpp((int)dlo(x), 0xB1, 0xF, 0xF, false),
                           (unsigned)__builtin_amdgcn_mov_dpp((int)dhi(x), 0xB1, 0xF, 0xF, false));
    x += y;
    const double z = dmake((unsigned)__builtin_amdgcn_mov_dpp((int)dlo(x), 0x4E, 0xF, 0xF, false),
                           (unsigned)__builtin_amdgcn_mov_dpp((int)dhi(x), 0x4E, 0xF, 0xF, false));
    return x + z;
}

// Value of lane `lane` (wave-uniform) in every lane.
__device__ __forceinline__ double bcast(double x, int lane) {
    return dmake((unsigned)__builtin_amdgcn_readlane((int)dlo(x), lane),
                 (unsigned)__builtin_amdgcn_readlane((int)dhi(x), lane));
}

// For a per-lane value x (lane l holding the entry of column l), the values
// of lanes c, 16 + c, 32 + c, 48 + c with c = l % 16 (the four 16-column
// blocks of column c), in every lane.
__device__ __forceinline__ void gather_cols(double x, double (&out)[4]) {
    const dpair a = pair16(x);      // rows (0, 1) or (2, 3) of my half
    const dpair e = pair32(a.even);  // rows 0 and 2
    const dpair o = pair32(a.odd);   // rows 1 and 3
    out[0] = e.even;
    out[1] = o.even;
    out[2] = e.odd;
    out[3] = o.odd;
}

// Full wavefront sum on VALU (DPP row rotations, then permlane swaps).  The
// value is exact in every lane but may differ in the last bit between
// lanes (each lane adds in its own order); use it from one lane only when
// bitwise agreement matters.
__device__ __forceinline__ double sum_wave_valu(double x) {
#define THO_ROR(v, c)                                                                   \
    dmake((unsigned)__builtin_amdgcn_mov_dpp((int)dlo(v), c, 0xF, 0xF, false),          \
          (unsigned)__builtin_amdgcn_mov_dpp((int)dhi(v), c, 0xF, 0xF, false))
    x += THO_ROR(x, 0x128);  // row_ror:8
    x += THO_ROR(x, 0x124);  // row_ror:4
    x += THO_ROR(x, 0x122);  // row_ror:2
    x += THO_ROR(x, 0x121);  // row_ror:1
#undef THO_ROR
    return sum_groups(x);
}

// Full wavefront sum.
__device__ __forceinline__ double sum_wave(double x) {
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

__device__ __forceinline__ double ldg(const double* p) { return __builtin_nontemporal_load(p); }

// K index of K-step s for lane group g in the MFMA row products X B whose X
// streams from HBM (the update A + V Z, the formation's V N): a pair of
// K-steps takes two adjacent columns and the four lane groups sit side by
// side, so that one 16-byte load per lane covers 64 contiguous bytes of each
// of 16 rows and two consecutive pairs a whole 128-byte line.  K must be a
// multiple of 8.
__host__ __device__ constexpr int rows_kidx(int s, int g) { return 8 * (s >> 1) + 2 * g + (s & 1); }

}  // namespace tho
