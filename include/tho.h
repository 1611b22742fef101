/*
 * tho.h -- C ABI of the two-stage Householder orthogonalization library
 * (libtho.so), hand-written HIP kernels for AMD gfx950 (MI355X).
 *
 * Problem (He & Shao, "On Two-Stage Householder Orthogonalization", §1):
 * given V (n x k0) with orthonormal columns and A (n x k), k0 + k << n, find
 * Q (n x k) with orthonormal columns, Q orthogonal to V, and R (k x k upper
 * triangular), S (k0 x k) such that
 *        [V, A] = [V, Q] [[I, S], [0, R]]          (eq. (4))
 * and [V, Q]^* [V, Q] = I.
 *
 * Conventions shared by every entry point
 *   - All matrices are DEVICE pointers, row-major with unit column stride and
 *     row stride ld (in elements), ld >= number of columns.  Element type is
 *     IEEE double (THO_F64) or interleaved (re, im) double pairs (THO_C128,
 *     the layout of std::complex<double> / torch.complex128).
 *   - The caller owns every buffer.  Inputs (V, A, ...) are read-only.
 *     Outputs (Q, R, S, ...) are fully overwritten; the strictly lower part
 *     of R is written as zero.  Outputs must not alias inputs or each other.
 *   - diag(R) is real and nonnegative and Q is scaled consistently (the
 *     phase convention used throughout; the paper uses QR variants with a
 *     nonnegative R diagonal for P, §3.2 and §6).
 *   - Work is enqueued on `stream` (a hipStream_t passed as void*; NULL is
 *     the default stream).  Calls return after enqueueing; they never
 *     synchronize the device and never allocate device memory (the
 *     workspace is caller-provided).  Calls with distinct workspaces may run
 *     concurrently.
 *   - Return value: 0 on success; -i when argument i (1-based) is invalid
 *     (LAPACK style: sizes, ld too small, NULL pointer, bad alignment, an
 *     output sharing elements with an input or another output);
 *     THO_E_WORKSPACE when ws_bytes is too small; THO_E_HIP when a HIP call
 *     failed (see tho_last_error()); THO_E_UNSUPPORTED for a valid but
 *     unimplemented combination.  Numerical conditions (non-finite input,
 *     a V that is not orthonormal) are not errors of the call: non-finite
 *     values propagate as NaN like LAPACK, and tho_two_stage reports them
 *     on request through a device info word (THO_CHECK_*, tho_get_info).
 */
#ifndef THO_H
#define THO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { THO_F64 = 0, THO_C128 = 1 } tho_dtype_t;

/* Choice of the unitary P of Algorithm 1 (§3.2), for the top k0 x k0 block
 * V_top of V:
 *   THO_P_QR     second choice (default; recommended in §6.2 and §7):
 *                V_top = Q1 R1, diag(R1) >= 0, P = -Q1, T = I + R1^* (lower
 *                triangular, kappa_2(T) < 2 sqrt(2) k0)
 *   THO_P_MLU    first choice: P diagonal (+-1), fixed during the modified
 *                LU factorization P - V_top = L U of Algorithm 2 [BDGJKN2015];
 *                T = U^* L^* P.  Not always stable: kappa_2(U) can be large
 *                (eq. (6), Table 4) and the loss of orthogonality grows with it
 *   THO_P_POLAR  third choice: polar decomposition V_top = Q2 M, P = -Q2,
 *                T = I + M (Hermitian positive definite, kappa_2(T) <= 2),
 *                solved by Cholesky; the polar factor comes from a one-sided
 *                Jacobi SVD of V_top in one workgroup
 * Each runs in one workgroup beside the first reduction over n rows.  The
 * complex path, the adjoint, the batched path, tho_hhqr_full and tho_bcgs use
 * THO_P_QR only (THO_E_UNSUPPORTED otherwise). */
typedef enum { THO_P_QR = 0, THO_P_MLU = 1, THO_P_POLAR = 2 } tho_pchoice_t;

/* Arithmetic of the four n x k0 x k panel products of Algorithm 1 (V^*A,
 * the update A + V Z, V^*Q_ and Q_ + V N).  Reflector generation, norms and
 * the T factors always stay FP64.  THO_PANEL_F32X2 splits each FP64 operand
 * into an FP32 hi + lo pair (three FP32 MFMA products, FP32 accumulation
 * inside each MFMA block, FP64 across blocks); THO_PANEL_BF16 rounds the
 * operands to BF16 (FP32 accumulation).  Reduced-precision panels lose
 * orthogonality of Q (to about 1e-8 and 1e-3 respectively) and on MI355X are
 * not faster than FP64 panels, whose Householder core dominates the time. */
typedef enum { THO_PANEL_F64 = 0, THO_PANEL_F32X2 = 1, THO_PANEL_BF16 = 2 } tho_panel_t;

/* Optional numerical-condition checks of tho_two_stage (opts->flags, OR of):
 *   THO_CHECK_FINITE  report a non-finite value in V or A (or produced by
 *                     overflow inside the method).  Costs one tiny kernel:
 *                     every element of V and A is a factor in the
 *                     reductions that form S and R (V^* A, the Householder
 *                     column norms), and IEEE products and sums keep NaN and
 *                     infinities non-finite (0 * Inf = NaN), so the check
 *                     scans the k0 x k + k x k outputs S and R.
 *   THO_CHECK_VORTH   report ||V^* V - I||_F > THO_VORTH_TOL (V is assumed
 *                     orthonormal, Algorithm 1's precondition; the loss of
 *                     orthogonality of Q grows with this distance, Theorem 1
 *                     and the remark after it).  Costs one extra split-n
 *                     Gram reduction over V (one more pass over V and
 *                     2 n k0^2 flops).
 * Results go to the info word (see tho_get_info), never to the return value:
 * the call still completes and the outputs are written. */
#define THO_CHECK_FINITE 1
#define THO_CHECK_VORTH  2
#define THO_VORTH_TOL    1e-10

/* Codes of the info word (0 = no condition detected).  When several
 * conditions hold, the smallest code is reported. */
#define THO_INFO_NONFINITE        1
#define THO_INFO_T_SINGULAR       2  /* reserved: no choice of P can give a singular T
                                        (the modified-LU pivots have modulus >= 1) */
#define THO_INFO_V_NOT_ORTHONORMAL 3

typedef struct {
    int32_t p_choice;   /* tho_pchoice_t */
    int32_t panel;      /* tho_panel_t   */
    int32_t flags;      /* THO_CHECK_* bits (tho_two_stage, tho_two_stage_noalloc); 0 elsewhere */
    int32_t reserved;
} tho_opts_t;

#define THO_E_WORKSPACE   (-100)
#define THO_E_HIP         (-101)
#define THO_E_UNSUPPORTED (-102)

/* Largest supported k0 and k (the k0 x k0 and k x k factorizations run
 * inside one workgroup).  THO_C128 supports k0 <= 64 and k <= 32
 * (THO_E_UNSUPPORTED beyond); reduced-precision panels and the batched
 * path are real (THO_F64) only. */
#define THO_MAX_K0 128
#define THO_MAX_K  64
#define THO_MAX_K0_C128 64
#define THO_MAX_K_C128  32

/* Bytes of device workspace tho_two_stage needs for these sizes (opts may be
 * NULL for defaults; p_choice and flags change the size).  Returns 0 or -i
 * like the other calls.  The first 256 bytes of the workspace hold the info
 * word of the last tho_two_stage call that used it (tho_get_info). */
int tho_two_stage_workspace(int32_t dtype, int64_t n, int64_t k0, int64_t k,
                            const tho_opts_t* opts, size_t* bytes);

/* Algorithm 1 of the paper (§3.1) with the choice of P in opts->p_choice
 * (§3.2; default the second choice):
 *   P = -Q1 where V_top = Q1 R1 (diag R1 >= 0), W = [P; 0] - V, T = I + R1^*,
 *   A <- (I - W T^{-*} W^*) A,  S = P^* A_top,  A_low = Q_ R (Householder),
 *   Q = (I - W T^{-1} W^*) [0; Q_].
 * In exact arithmetic (Q, R, S) do not depend on the choice of P; in
 * floating point the first choice can lose orthogonality (Table 4).
 * Arguments: 1 dtype, 2 n, 3 k0, 4 k, 5 V (n x k0), 6 ldv, 7 A (n x k),
 * 8 lda, 9 Q (n x k, out), 10 ldq, 11 R (k x k, out), 12 ldr, 13 S (k0 x k,
 * out), 14 lds, 15 opts (NULL = defaults), 16 ws, 17 ws_bytes, 18 stream.
 * Requires n >= k0 + k, 0 <= k0 <= THO_MAX_K0, 0 <= k <= THO_MAX_K.
 * k0 == 0 computes a plain Householder QR of A; k == 0 is a no-op.  V is
 * assumed orthonormal; if it is not, Q loses orthogonality in proportion to
 * ||V^*V - I|| (Theorem 1 and the remark after it) -- not an error.
 * A rank-deficient A is not an error: Q is still orthonormal and orthogonal
 * to V (§1, the reason for Householder-QR as the intra-block step). */
int tho_two_stage(int32_t dtype, int64_t n, int64_t k0, int64_t k,
                  const void* V, int64_t ldv, const void* A, int64_t lda,
                  void* Q, int64_t ldq, void* R, int64_t ldr, void* S, int64_t lds,
                  const tho_opts_t* opts, void* ws, size_t ws_bytes, void* stream);

/* The info word of the last tho_two_stage call that used workspace `ws`
 * (NULL: the calling device's static scratch of tho_two_stage_noalloc),
 * as a THO_INFO_* code, 0 when no condition was detected or no check was
 * requested.  Every tho_two_stage call with k > 0 rewrites the word on its
 * stream; read it only after that stream has been synchronized (the call
 * copies 4 bytes device to host with hipMemcpy).  Arguments: 1 ws (device),
 * 2 host_info (host, out).  Returns 0, -2 for a NULL host_info, THO_E_HIP,
 * or THO_E_UNSUPPORTED for ws = NULL before any tho_two_stage_noalloc call
 * on the device. */
int tho_get_info(const void* ws, int32_t* host_info);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * tho_two_stage without a workspace argument.  Its work buffer is a
 * library-owned static device array of THO_NOALLOC_SCRATCH_BYTES bytes per
 * GPU, held from the first call on that GPU until the process ends; the
 * call allocates no device memory (hipMalloc, hipFree or any allocating
 * library routine).  The first call on a device and host thread also
 * creates that thread's side stream and two events (no device memory).
 * Arguments 1-15 and the result are those of tho_two_stage (arguments 1-15)
 * and its `stream` (argument 16); sizes whose tho_two_stage_workspace exceeds
 * THO_NOALLOC_SCRATCH_BYTES are rejected with THO_E_WORKSPACE before any
 * work is enqueued (for FP64 that admits, e.g., n = 2^20 with k0 = 64,
 * k = 32).  Every call on one GPU shares that GPU's array and the array keeps
 * the last call's contents (each call initialises what it reads):
 * calls that overlap in time on the same GPU -- on different streams or from
 * different host threads -- race and give wrong results; serialize them. */
#define THO_NOALLOC_SCRATCH_BYTES (256u << 20)
int tho_two_stage_noalloc(int32_t dtype, int64_t n, int64_t k0, int64_t k,
                          const void* V, int64_t ldv, const void* A, int64_t lda,
                          void* Q, int64_t ldq, void* R, int64_t ldr, void* S, int64_t lds,
                          const tho_opts_t* opts, void* stream);

/* Householder QR of the whole matrix [V, A] (the baseline the method is
 * compared with in §6: V's columns are factored too, nothing assumes V is
 * orthonormal).  Computed as the block Householder QR of Algorithm 4 over
 * column panels of at most 64: the first panel of V by the chunked
 * Householder QR, every later panel (the rest of V, then A) by the
 * generalized Householder step of Algorithm 1 against the computed Q of the
 * earlier panels.  With [V, A] = Q_B R_B (nonnegative diag R_B) it returns
 * Q = Q_B[:, k0:], R = R_B[k0:, k0:], S = R_B[:k0, k0:] -- the layout of
 * eq. (4).  Arguments as tho_two_stage; THO_F64 only.  The workspace holds
 * the n x k0 basis of V's panels. */
int tho_hhqr_full_workspace(int32_t dtype, int64_t n, int64_t k0, int64_t k, const tho_opts_t* opts, size_t* bytes);
int tho_hhqr_full(int32_t dtype, int64_t n, int64_t k0, int64_t k,
                  const void* V, int64_t ldv, const void* A, int64_t lda,
                  void* Q, int64_t ldq, void* R, int64_t ldr, void* S, int64_t lds,
                  const tho_opts_t* opts, void* ws, size_t ws_bytes, void* stream);

/* Block Householder-QR (Algorithm 4, §6.1): A = [A_1, ..., A_p] (n x K,
 * block widths kb[0..p-1], each in [1, THO_MAX_K], K = sum of widths <= n)
 * factored block by block as block Krylov methods produce the blocks:
 * A = Q R with Q^* Q = I (n x K) and R upper triangular (K x K,
 * nonnegative diagonal).  Block i is orthogonalized against the basis
 * [Q_1, ..., Q_{i-1}] of the blocks before it by a generalized Householder
 * transformation and its bottom rows are factored by Householder QR, so the
 * basis may be far wider than THO_MAX_K0.  The transformation of block i
 * uses the block-diagonal P = diag(P_1, ..., P_{i-1}), P_j by opts->p_choice
 * from block j's own bottom basis, which makes it the product of one
 * Algorithm 1 transformation per earlier block (each a pass over the rows
 * below that block); Q and R do not depend on P in exact arithmetic.
 * Real FP64 only.
 * tho_block_householder: arguments 1 dtype, 2 n, 3 nblocks, 4 kb (host
 * array), 5 A (n x K), 6 lda, 7 Q (n x K, out), 8 ldq, 9 R (K x K, out,
 * strictly lower part written as 0), 10 ldr, 11 opts (panel and flags must
 * be default), 12 ws, 13 ws_bytes, 14 stream.  Q and R must not overlap A
 * or each other.
 * tho_block_householder_step appends one block to a basis kept in the
 * workspace (the append operation of a block Krylov loop): block i
 * (0-based) with widths kb[0..i]; call it for i = 0, 1, 2, ... with the
 * same Q, R and workspace.  Arguments 1 dtype, 2 n, 3 i, 4 kb, 5 kmax (the
 * largest total width the workspace is sized for), 6 A_i (n x k_i), 7 lda,
 * 8 Q (n x kmax: columns of earlier blocks as written by earlier steps;
 * block i's columns are written), 9 ldq, 10 R (written: rows
 * 0 .. c_i + k_i - 1 of block column i, c_i = kb[0] + ... + kb[i-1]),
 * 11 ldr, 12 opts, 13 ws, 14 ws_bytes, 15 stream.
 * tho_block_householder_workspace(dtype, n, kmax, opts, bytes) sizes the
 * workspace of either call for total widths up to kmax (it holds the n x kmax
 * bottom bases of the blocks).  Errors as elsewhere (-i, THO_E_*). */
int tho_block_householder_workspace(int32_t dtype, int64_t n, int64_t kmax, const tho_opts_t* opts, size_t* bytes);
int tho_block_householder(int32_t dtype, int64_t n, int32_t nblocks, const int64_t* kb, const void* A, int64_t lda,
                          void* Q, int64_t ldq, void* R, int64_t ldr, const tho_opts_t* opts, void* ws,
                          size_t ws_bytes, void* stream);
int tho_block_householder_step(int32_t dtype, int64_t n, int32_t i, const int64_t* kb, int64_t kmax, const void* Ai,
                               int64_t lda, void* Q, int64_t ldq, void* R, int64_t ldr, const tho_opts_t* opts,
                               void* ws, size_t ws_bytes, void* stream);

/* Two-stage orthogonalization in the weighted inner product
 * <x, y>_B = x^* diag(b) y (Algorithm 3, §5, with a diagonal positive
 * definite B = diag(b)): given V with V^* B V = I and A, returns Q, R, S with
 * [V, A] = [V, Q] [[I, S], [0, R]] and [V, Q]^* B [V, Q] = I.  With
 * D = diag(sqrt(b)), the generalized Householder transformation of
 * Theorem 4 is D^{-1} H~ D (H~ the Euclidean one for the scaled data) and the
 * initial B-orthonormal basis of §5 is D^{-1} [I; 0], so the method is
 * Algorithm 1 on (D V, D A) followed by Q = D^{-1} Q~: the rows are scaled in
 * streaming kernels around tho_two_stage (opts as there, including
 * p_choice and the THO_CHECK_* flags, which then apply to D V and D A).
 * Arguments: 1 dtype, 2 n, 3 k0, 4 k, 5 b (n doubles, device, all > 0; a
 * nonpositive entry gives NaN, reported by THO_CHECK_FINITE), 6-15 V .. lds as
 * arguments 5-14 of tho_two_stage, 16 opts, 17 ws, 18 ws_bytes, 19 stream.
 * The workspace holds tho_two_stage's own first (tho_get_info(ws) reads the
 * info word as for tho_two_stage) and then scaled copies of V and A.  A
 * general (non-diagonal) B is not supported. */
int tho_two_stage_weighted_workspace(int32_t dtype, int64_t n, int64_t k0, int64_t k, const tho_opts_t* opts,
                                     size_t* bytes);
int tho_two_stage_weighted(int32_t dtype, int64_t n, int64_t k0, int64_t k, const double* b,
                           const void* V, int64_t ldv, const void* A, int64_t lda,
                           void* Q, int64_t ldq, void* R, int64_t ldr, void* S, int64_t lds,
                           const tho_opts_t* opts, void* ws, size_t ws_bytes, void* stream);

/* Block classical Gram-Schmidt, the baseline of eq. (1) and Table 1:
 * `rounds` rounds, each running `proj` projections
 *     C = V^T X,  X <- X - V C,  S_r <- S_r + C          (BQR-1)
 * followed by one Householder QR X = Q_r R_r (BQR-2, the same chunked
 * Householder QR as tho_two_stage, nonnegative diag R_r).  Round 1 starts
 * from X = A, later rounds from the previous Q.  Outputs satisfy
 * A ~ V S + Q R with S = S_1 + S_2 R_1 + S_3 R_2 R_1 + ..., R = R_r ... R_1.
 * Table 1's rows are (proj, rounds) = (1,1), (2,1), (1,2), (3,1), (1,3).
 * Arguments 1-14 as tho_two_stage; 15 proj (1..8), 16 rounds (1..8),
 * 17 opts (panel must be THO_PANEL_F64), 18 ws, 19 ws_bytes, 20 stream.
 * THO_F64 only (THO_E_UNSUPPORTED otherwise).  Unlike the two-stage method,
 * the orthogonality of Q is only as good as the conditioning of [V, A]
 * allows (Table 1): this is the comparison baseline, not a robust method. */
int tho_bcgs_workspace(int32_t dtype, int64_t n, int64_t k0, int64_t k, int32_t proj, int32_t rounds,
                       const tho_opts_t* opts, size_t* bytes);
int tho_bcgs(int32_t dtype, int64_t n, int64_t k0, int64_t k,
             const void* V, int64_t ldv, const void* A, int64_t lda,
             void* Q, int64_t ldq, void* R, int64_t ldr, void* S, int64_t lds,
             int32_t proj, int32_t rounds,
             const tho_opts_t* opts, void* ws, size_t ws_bytes, void* stream);

/* Adjoint (reverse-mode gradient) of the map (V, A) -> (Q, R, S) that
 * tho_two_stage computes, real FP64 and complex128 (k0 <= 64, k <= 32 for
 * complex).  The paper does not treat
 * differentiation; this is the exact adjoint of the steps of Algorithm 1
 * (second choice of P) taken in reverse order, with the thin-QR adjoint
 * X_bar = (Q_bar + Q copyltu(R R_bar^T - Q_bar^T Q)) R^{-T} for the QR of
 * the bottom block and for the square QR of V_top.  For a scalar loss l with
 * gQ = dl/dQ, gR = dl/dR (only its upper triangle is used) and gS = dl/dS,
 * it returns dV = dl/dV and dA = dl/dA, V and A taken as unconstrained
 * matrices.  Q and R must be the outputs of tho_two_stage for (V, A); the
 * WY factors are recomputed from V, A, Q (never stored), using W^T Q = -T^T N
 * which holds for orthonormal V.  Complex data: the loss is
 * l = Re<gQ, Q> + Re<gR, R> + Re<gS, S> with <X, Y> = sum conj(X) Y, and dV,
 * dA satisfy dl = Re<dV, dV_dir> + Re<dA, dA_dir> (PyTorch's convention);
 * the steps are the same with conjugate transposes, and the thin-QR adjoint
 * uses copyltu(M) = tril(M, -1) + tril(M, -1)^H + Re(diag M).
 * Arguments: 1 dtype, 2 n, 3 k0, 4 k, 5 V, 6 ldv, 7 A, 8 lda,
 * 9 Q, 10 ldq, 11 R, 12 ldr, 13 gQ (n x k), 14 ldgq, 15 gR (k x k),
 * 16 ldgr, 17 gS (k0 x k, may be NULL for zero), 18 ldgs, 19 dV (n x k0,
 * out), 20 lddv, 21 dA (n x k, out), 22 ldda, 23 opts, 24 ws, 25 ws_bytes,
 * 26 stream.  dV and dA are fully overwritten and must not alias inputs.
 * R must be nonsingular (the QR adjoint divides by diag R). */
int tho_two_stage_backward_workspace(int32_t dtype, int64_t n, int64_t k0, int64_t k, const tho_opts_t* opts,
                                     size_t* bytes);
int tho_two_stage_backward(int32_t dtype, int64_t n, int64_t k0, int64_t k,
                           const void* V, int64_t ldv, const void* A, int64_t lda,
                           const void* Q, int64_t ldq, const void* R, int64_t ldr,
                           const void* gQ, int64_t ldgq, const void* gR, int64_t ldgr,
                           const void* gS, int64_t ldgs,
                           void* dV, int64_t lddv, void* dA, int64_t ldda,
                           const tho_opts_t* opts, void* ws, size_t ws_bytes, void* stream);

/* ---- Batched problems (many independent (V, A) pairs of uneven sizes).
 * Each problem runs Algorithm 1 (second choice of P) exactly as
 * tho_two_stage computes it, except that its Householder QR is one chunk of
 * tiles (no reduction tree): the whole problem is processed by one
 * workgroup of a single persistent kernel, which takes problems longest
 * first from a device work counter.  Plan creation validates the problems,
 * lays out each problem's part of the caller's workspace, autotunes the tile
 * height (128 or 256 rows) and the number of persistent workgroups by timing
 * them on the batch itself (cached per batch signature and device for the
 * life of the process and, when the environment variable THO_TUNE_CACHE
 * names a file, in that file across processes: one text line per choice,
 * read at the first plan creation and appended after each new tuning), and
 * captures the launches into a HIP graph.  The plan binds the
 * problem pointers and the workspace: tho_batched_run replays the graph on
 * `stream` and may be called any number of times while the buffers live.
 * Plan creation allocates small device descriptor arrays (freed by
 * tho_plan_destroy), synchronizes with `stream` once, and runs the batch a
 * few times while tuning (outputs are overwritten).  Real FP64 only,
 * default options only. */
#define THO_BATCHED_MAX_K0 64

typedef struct {
    int64_t n, k0, k;      /* n >= k0 + k, 0 <= k0 <= 64, 0 <= k <= 64 */
    const void* V; int64_t ldv;
    const void* A; int64_t lda;
    void* Q; int64_t ldq;
    void* R; int64_t ldr;
    void* S; int64_t lds;
} tho_problem_t;

typedef struct tho_plan_s* tho_plan_t;

/* Workspace bytes for a batch (arguments: 1 count, 2 problems (host array),
 * 3 opts, 4 bytes out).  An invalid problem returns -2 and names it in
 * tho_last_error(). */
int tho_batched_workspace(int32_t count, const tho_problem_t* problems, const tho_opts_t* opts, size_t* bytes);
/* Arguments: 1 count, 2 problems (host array, copied), 3 ws, 4 ws_bytes,
 * 5 opts, 6 stream, 7 plan out. */
int tho_batched_plan_create(int32_t count, const tho_problem_t* problems, void* ws, size_t ws_bytes,
                            const tho_opts_t* opts, void* stream, tho_plan_t* plan);
int tho_batched_run(tho_plan_t plan, void* stream);
/* Autotuner result: tile height in rows, persistent workgroups, and the best
 * measured batch time in ms (0 when the choice came from the cache). */
int tho_batched_plan_info(tho_plan_t plan, int32_t* tile_rows, int32_t* grid, double* tuned_ms);
int tho_plan_destroy(tho_plan_t plan);

/* Benchmark instrumentation (not needed for normal use).
 * tho_profile_enable(1) makes every later call record a pair of hipEvents on
 * its stream around each kernel it launches.  tho_profile_collect() waits
 * for the recorded events, folds their elapsed times into per-kernel-name
 * totals and returns the number of distinct names (or a negative error);
 * tho_profile_get(i, ...) reads entry i (name into a caller buffer of
 * name_len bytes, accumulated milliseconds, number of launches);
 * tho_profile_reset() clears the totals.  Process-global, thread-safe. */
int tho_profile_enable(int on);
int tho_profile_collect(void);
int tho_profile_reset(void);
int tho_profile_get(int i, char* name, int name_len, double* total_ms, int64_t* launches);

/* Message for the last THO_E_HIP / argument error on this thread. */
const char* tho_last_error(void);

/* Static description of an error code. */
const char* tho_strerror(int code);

/* Library version string. */
const char* tho_version(void);

#ifdef __cplusplus
}
#endif

#endif /* THO_H */
