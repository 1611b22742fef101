// Host-side declarations of the kernel launchers inside libtho (not part of
// the public C ABI; see include/tho.h for that).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tho {

// Tile geometry of the tall-skinny Householder kernels: a workgroup of
// LEAF_WAVES wavefronts owns a tile of tsqr_tile_rows(kp) rows held in
// registers (16-row MFMA blocks per wavefront).
constexpr int LEAF_WAVES = 4;
int tsqr_tile_rows(int kp);

// Arguments of one level of the chunked tall-skinny QR (leaf) and of the
// matching Q formation (form).  Level 0 works on the bottom n - k0 rows of A
// (forming A + V Z on the fly) and stores Householder vectors into the Q
// output; levels >= 1 work in place on the stacked R factors of the level
// below.
struct TsqrLevel {
    int64_t m;        // rows of this level's matrix
    int k;            // columns (<= KP)
    int nchunk;       // chunks (one workgroup each)
    int maxtiles;     // tile slots reserved per chunk
    const double* X;  // input rows (leaf); ld ldx
    int64_t ldx;
    double* Y;        // Householder vectors out (leaf) / Q rows out (form); ld ldy
    int64_t ldy;
    // level 0 with k0 > 0 only
    const double* V;  // bottom rows of V; ld ldv
    int64_t ldv;
    int k0;
    const double* Z;  // K0P x KP Z of the update of A, in B-operand order (k_permute_b)
    double* Nc;       // per chunk KP x K0P: Q_chunk^T V_chunk (leaf output)
    const double* Nglob;  // K0P x KP N = T^{-1} G, in B-operand order (form input)
    // reduced-precision panels: Z and N packed by launch_pack_b_lowp
    const void* Zlp;
    const void* Nlp;
    // per-tile storage
    double* tau;      // [nchunk * maxtiles][KP]
    double* Tt;       // [nchunk * maxtiles][KP * KP]
    // leaf: R factor of chunk c goes to rows c*k .. c*k+k-1 of Rnext (ld ldrn)
    double* Rnext;
    int64_t ldrn;
    // form: G_c of chunk c is rows c*gstride .. of Gin (ld ldg)
    const double* Gin;
    int64_t ldg;
    int64_t gstride;
    // two-pass formation of level 0: per chunk KP x KP, the block C that
    // reaches the chunk's first tile (row-major, zero outside k x k)
    double* Cfin;
};

// part[blk] = X^T [Y0 Y1 Y2] over the block's rows for three matrices of q
// columns each: (16 mt) x (48 nb) per block, the Y_i blocks side by side.
hipError_t launch_xty3_partial(int mt, int nb, int64_t nrows, const double* X, int64_t ldx, int p, const double* Y0,
                               int64_t ld0, const double* Y1, int64_t ld1, const double* Y2, int64_t ld2, int q,
                               int nblk, int64_t rows_per_blk, double* part, hipStream_t st);
hipError_t launch_xty_partial(int mt, int nt, int64_t nrows, const double* X, int64_t ldx, int p,
                              const double* Y, int64_t ldy, int q, int nblk, int64_t rows_per_blk,
                              double* part, hipStream_t st);
hipError_t launch_reduce_parts(int nparts, int64_t elems, const double* part, double* out,
                               hipStream_t st);
hipError_t launch_small_gemm(int M, int N, int K, double alpha, const double* A, int64_t lda, int ta,
                             const double* B, int64_t ldb, int tb, double beta, const double* C,
                             int64_t ldc, double* D, int64_t ldd, hipStream_t st);
hipError_t launch_trsm_lower(int n, int m, const double* L, int64_t ldl, int trans, double* B,
                             int64_t ldb, hipStream_t st);
hipError_t launch_qr_top(int n, const double* Vt, int64_t ldv, double* P, double* T, hipStream_t st);
// First and third choices of P for the n x n top block (n <= 128), one
// workgroup each (k_pchoice.hip).  launch_mlu_top: P = diag, F1 = P L,
// F2 = U^T with P - V_top = L U (Algorithm 2).  launch_polar_top: P = -Q2
// and C = chol(I + M) for V_top = Q2 M; ws holds pchoice_ws_doubles(n).
hipError_t launch_mlu_top(int n, const double* Vt, int64_t ldv, double* P, double* F1, double* F2, hipStream_t st);
hipError_t launch_polar_top(int n, const double* Vt, int64_t ldv, double* P, double* C, double* ws, hipStream_t st);
size_t pchoice_ws_doubles(int n);

// Y = diag(sqrt(b)) X (inv = 0) or diag(1 / sqrt(b)) X (inv = 1), n rows of
// w doubles (k_weighted.hip).
hipError_t launch_row_scale(int64_t n, int w, const double* b, int inv, const double* X, int64_t ldx, double* Y,
                            int64_t ldy, hipStream_t st);

// Numerical-condition checks (k_checks.hip): the info word is INT_MAX until
// a condition lowers it (atomicMin) to its code.
hipError_t launch_info_reset(int* info, hipStream_t st);
hipError_t launch_check_finite(int k0, int k, int cplx, const double* S, int64_t lds, const double* R, int64_t ldr,
                               int* info, hipStream_t st);
// G0, G1: column blocks 0..63 and 64.. of the Gram (ld ld0, ld1).
hipError_t launch_vorth_check(int k0, int cplx, const double* G0, int ld0, const double* G1, int ld1, double tol,
                              int* info, hipStream_t st);
hipError_t launch_finish_r(int k, int KP, const double* Rin, int64_t ldri, double* Rout, int64_t ldr,
                           double* G0, hipStream_t st);
hipError_t launch_permute_b(int K0P, int KP, const double* src, double* dst, hipStream_t st);
hipError_t launch_chunk_prod(int nchunk, int K0P, int KP, int k, const double* Nc, const double* Gbase,
                             int64_t ldg, int64_t grow_stride, double* prod, hipStream_t st);

// Elementwise small-matrix helper (M x N):
//   D = a op(X) + b op(Y) + c I, then masked by `mode`
// op(.) transposes when tx / ty; mode 0 none, 1 lower (j <= i kept),
// 2 upper (j >= i kept), 3 copyltu (lower part mirrored to the upper).
// X or Y may be null (term skipped).  D must not alias X or Y when a
// transpose or mode 3 is used.
hipError_t launch_small_ew(int M, int N, double a, const double* X, int64_t ldx, int tx, double b, const double* Y,
                           int64_t ldy, int ty, double c, int mode, double* D, int64_t ldd, hipStream_t st);

// ---- complex path (k_complex.hip): interleaved (re, im) doubles
struct dcplx {
    double re, im;
};
// One level of the complex chunked TSQR (leaf) / formation (form); the same
// roles as TsqrLevel without the fused V products.
struct ZLevel {
    int64_t m;
    int k, nchunk, maxtiles, pad;
    const dcplx* X;
    int64_t ldx;
    dcplx* Y;
    int64_t ldy;
    dcplx* Tt;     // [nchunk * maxtiles][KP * KP]
    dcplx* Rnext;  // chunk R factors, rows c*k .., ld ldrn
    int64_t ldrn;
    const dcplx* Gin;
    int64_t ldg;
    int64_t gstride;
};
int ztsqr_tile_rows(int kp);
hipError_t launch_zleaf(int kp, const ZLevel& L, hipStream_t st);  // kp in {16, 32}
// Level 0 of the complex chunked QR in registers (k_zleaf.hip) with the
// update A + V Z fused in and the chunk products M_c = Q_chunk^H V_chunk
// (KP x K0P each, into Nc); outputs as launch_zleaf.  k0p 0 (no V term), 16,
// 32 or 64; tiles of zleaf_rt_tile_rows(kp) = ztsqr_tile_rows(kp) rows.
struct ZRLevel {
    int64_t m;
    int k, k0, nchunk, maxtiles;
    const dcplx* X;
    int64_t ldx;
    dcplx* Y;
    int64_t ldy;
    const dcplx* V;
    int64_t ldv;
    const dcplx* Zp;  // Z in B-operand order (launch_zpermute_b)
    dcplx* Tt;
    dcplx* Rnext;
    int64_t ldrn;
    dcplx* Nc;        // [nchunk][KP * K0P]
};
int zleaf_rt_tile_rows(int kp);
hipError_t launch_zleaf_rt(int kp, int k0p, const ZRLevel& L, hipStream_t st);
hipError_t launch_zpermute_b(int k0p, int kp, int k0, int k, const dcplx* Z, int64_t ldz, dcplx* out, hipStream_t st);
// Two-pass formation of complex level 0: the per-chunk k x k recurrence
// (overwrites each T_t with -K_t in B-operand order, fills Cfin), then every
// tile's rows of Q = [C; 0] - Y_t K_t + V_t N (Np: N in B-operand order).
hipError_t launch_zkchain(int kp, const ZLevel& L, dcplx* Cfin, hipStream_t st);
hipError_t launch_zrows0(int kp, int k0p, const ZLevel& L, const dcplx* Cfin, const dcplx* V, int64_t ldv, int k0,
                         const dcplx* Np, hipStream_t st);
// out_c = M_c^H G_c per chunk (k0p x kp complex each, zero-padded)
hipError_t launch_zchunk_prod(int nchunk, int k0, int k, int kp, int k0p, const dcplx* M, const dcplx* G, int64_t ldg,
                              int64_t gstride, dcplx* out, hipStream_t st);
hipError_t launch_zform(int kp, const ZLevel& L, hipStream_t st);
hipError_t launch_zqr_top(int n, const void* Vt, int64_t ldv, void* P, void* T, hipStream_t st);  // n <= 64
// D = alpha op(A) op(B) + beta C (op: 0 none, 1 transpose, 2 conjugate transpose)
hipError_t launch_zgemm(int M, int N, int K, double ar, double ai, const void* A, int64_t lda, int opa, const void* B,
                        int64_t ldb, int opb, double br, double bi, const void* C, int64_t ldc, void* D, int64_t ldd,
                        hipStream_t st);
// In-place solve with lower-triangular L: mode 0 L X = B, mode 2 L^H X = B.
hipError_t launch_ztrsm(int n, int m, const void* L, int64_t ldl, int mode, void* B, int64_t ldb, hipStream_t st);
// out = sign * X^H Y from the real-view reduction Cr = X_ri^T Y_ri (2p x 2q).
hipError_t launch_zcombine(int p, int q, const double* Cr, int64_t ldc, double sign, void* out, int64_t ldo,
                           hipStream_t st);
// Real 2 x 2 block form (2p x 2q, ld 2q) of sign * B (p x q complex).
hipError_t launch_zexpand(int p, int q, const void* B, int64_t ldb, double sign, double* dst, hipStream_t st);
hipError_t launch_zfinish_r(int k, int KP, const void* Rin, int64_t ldri, void* Rout, int64_t ldr, void* G0,
                            hipStream_t st);
hipError_t launch_zcopy(int64_t M, int N, const void* src, int64_t lds, void* dst, int64_t ldd, hipStream_t st);
// D = a op(X) + b op(Y) + c I, complex, masked (mode 1 lower, 2 upper, 3 copyltu).
hipError_t launch_zsmall_ew(int M, int N, double a, const void* X, int64_t ldx, int opx, double b, const void* Y,
                            int64_t ldy, int opy, double c, int mode, void* D, int64_t ldd, hipStream_t st);

// One problem of the batched path (k_batched.hip): inputs/outputs as in
// tho_two_stage plus its own workspace pieces (all device pointers).
struct BatchedInst {
    int64_t n;
    int k0, k, K0P, pad;
    const double* V;
    const double* A;
    double *Q, *R, *S;
    int64_t ldv, lda, ldq, ldr, lds;
    double *Pm, *Tm;        // k0 x k0 (ld k0): P and T
    double *Zperm, *Nperm;  // K0P x KP in B-operand order
    double* Nc;             // KP x K0P: N_c^T from the leaf
    double *Rtop, *G0;      // KP x KP
};
int batched_tile_rows(int kp, int rbo);
hipError_t launch_zero_ints(int* p, int n, hipStream_t st);
// Persistent launch over `count` problems of one (kp, k0p) class in the
// order `order` (kp in {16, 32, 64}, k0p in {0, 16, 32, 64}, rbo = 16-row
// blocks per wavefront of a tile: 2 or 4; kp = 64 takes 2 only).
hipError_t launch_batched(int kp, int k0p, int rbo, const BatchedInst* insts, const TsqrLevel* levels,
                          const int* order, int count, int* counter, int grid, hipStream_t st);

// Row-streaming panel product Out = X + sum_t Y_t B_t (k_stream.hip).
// X may be NULL (taken as 0) and may alias Out; q <= 128 output columns;
// each B_t is p_t x q packed by launch_pack_b with kpad_t (multiple of 16,
// >= p_t) rows and rows_gemm_qp(q) columns.
struct RowsTerm {
    const double* Y;
    int64_t ldy;
    int p;
    int kpad;
    const double* B;
};
struct RowsGemm {
    static constexpr int MAXT = 4;
    int64_t nrows;
    const double* X;
    int64_t ldx;
    double* Out;
    int64_t ldo;
    int q;
    int nterm;
    RowsTerm t[MAXT];
};
int rows_gemm_qp(int q);
hipError_t launch_rows_gemm(const RowsGemm& g, hipStream_t st);
// dst = scale * op(src) (p x q; op = transpose if trans) in B-operand order,
// zero padded to kpad x qp.
hipError_t launch_pack_b(int p, int q, const double* src, int64_t lds, int trans, double scale, int kpad, int qp,
                         double* dst, hipStream_t st);

// kp in {16, 32, 64}; k0p in {0, 16, 32, 64, 128} (0: no V term); panel
// 0 = FP64, 1 = FP32 hi + lo, 2 = BF16 for the V products (k0p > 0 only).
hipError_t launch_tsqr_leaf(int kp, int k0p, int panel, const TsqrLevel& L, hipStream_t st);
// Levels above 0 (no V term): factorization and formation with one
// workgroup of eight wavefronts per chunk, tiles of tsqr_tile_rows_up(kp).
int tsqr_tile_rows_up(int kp);
hipError_t launch_tsqr_leaf_up(int kp, const TsqrLevel& L, hipStream_t st);
hipError_t launch_tsqr_form_up(int kp, const TsqrLevel& L, hipStream_t st);
// Two-pass formation of level 0: the per-chunk recurrence of the k x k
// blocks (overwrites each T_t with -K_t and fills Cfin), then every tile's
// rows of Q independently.
hipError_t launch_tsqr_kchain(int kp, const TsqrLevel& L, hipStream_t st);
hipError_t launch_tsqr_rows(int kp, int k0p, int panel, const TsqrLevel& L, hipStream_t st);

// Reduced-precision panels (k_lowp.hip): C = X^T Y with FP32 hi + lo or
// BF16 products (same layout as launch_xty_partial), and the packing of a
// dense K0P x KP FP64 matrix into the B-operand order of the fused kernels.
hipError_t launch_xty_lowp(int panel, int mt, int nt, int64_t nrows, const double* X, int64_t ldx, int p,
                           const double* Y, int64_t ldy, int q, int nblk, int64_t rows_per_blk, double* part,
                           hipStream_t st);
size_t lowp_pack_bytes(int panel, int K0P, int KP);
hipError_t launch_pack_b_lowp(int panel, int K0P, int KP, const double* src, void* dst, hipStream_t st);

}  // namespace tho
