// Two-stage orthogonalization in a weighted inner product (Algorithm 3, §5,
// with B = diag(b), b > 0).  With B = D^2, D = diag(sqrt(b)), the
// generalized Householder transformation of Theorem 4 for (X, Y) is
// D^{-1} H~ D with H~ the Euclidean one for (D X, D Y), and the initial
// B-orthonormal basis of §5 is D^{-1} [I; 0]: Algorithm 3 is Algorithm 1 on
// (D V, D A) with Q = D^{-1} Q~.  The rows are scaled in streaming kernels
// around tho_two_stage, which does the rest.
#include <algorithm>

#include "tho_host.h"

using namespace tho;

namespace {

struct WPlan {
    double *Vs, *As;
    size_t head, bytes;
};

// tho_two_stage's own workspace first (so that its info word is at the
// start of the caller's workspace), then scaled copies of V and A (w doubles
// per element).
int wplan(int32_t dtype, int64_t n, int64_t k0, int64_t k, const tho_opts_t* opts, void* ws, WPlan& P) {
    const int w = dtype == THO_C128 ? 2 : 1;
    size_t tb = 0;
    int rc = tho_two_stage_workspace(dtype, n, k0, k, opts, &tb);
    if (rc) return rc;
    P.head = (tb + 255) & ~(size_t)255;
    Carve cv(ws ? (char*)ws + P.head : nullptr);
    P.Vs = cv.take((size_t)n * std::max<int64_t>(k0, 1) * w);
    P.As = cv.take((size_t)n * std::max<int64_t>(k, 1) * w);
    P.bytes = P.head + cv.bytes();
    return 0;
}

}  // namespace

extern "C" {

int tho_two_stage_weighted_workspace(int32_t dtype, int64_t n, int64_t k0, int64_t k, const tho_opts_t* opts,
                                     size_t* bytes) {
    int rc = check_common(dtype, n, k0, k);
    if (rc) return rc;
    if (!bytes) return set_err(-6, "bytes must not be NULL");
    if (k == 0) { *bytes = 0; return 0; }
    WPlan P;
    if ((rc = wplan(dtype, n, k0, k, opts, nullptr, P))) return rc;
    *bytes = P.bytes;
    return 0;
}

int tho_two_stage_weighted(int32_t dtype, int64_t n, int64_t k0, int64_t k, const double* b, const void* V,
                           int64_t ldv, const void* A, int64_t lda, void* Q, int64_t ldq, void* R, int64_t ldr,
                           void* S, int64_t lds, const tho_opts_t* opts, void* ws, size_t ws_bytes, void* stream) {
    int rc = check_common(dtype, n, k0, k);
    if (rc) return rc;
    if (k == 0) return 0;
    if (!b) return set_err(-5, "b is NULL");
    if ((uintptr_t)b & 7) return set_err(-5, "b must be 8-byte aligned");
    if ((rc = check_io(k0, k, V, ldv, A, lda, Q, ldq, R, ldr, S, lds))) return rc - 1;  // arguments shift by one
    const int w = dtype == THO_C128 ? 2 : 1;
    if ((rc = check_alias(n, k0, k, 8 * w, V, ldv, A, lda, Q, ldq, R, ldr, S, lds))) return rc - 1;
    // b (n doubles) must not share memory with an output (counted in doubles)
    if (blocks_overlap(Q, n, w * k, w * ldq, b, 1, n, n, 8) || blocks_overlap(R, k, w * k, w * ldr, b, 1, n, n, 8) ||
        (k0 > 0 && blocks_overlap(S, k0, w * k, w * lds, b, 1, n, n, 8)))
        return set_err(-5, "b overlaps an output");
    if (!ws) return set_err(-17, "workspace is NULL");
    WPlan P;
    if ((rc = wplan(dtype, n, k0, k, opts, nullptr, P))) return rc;
    if (ws_bytes < P.bytes) return set_err(THO_E_WORKSPACE, "workspace too small");
    wplan(dtype, n, k0, k, opts, ws, P);
    hipStream_t st = (hipStream_t)stream;
    const int64_t k0w = std::max<int64_t>(k0, 1);
    // D V and D A
    if (k0 > 0) PROF("row_scale", st, launch_row_scale(n, (int)(w * k0), b, 0, (const double*)V, w * ldv, P.Vs, w * k0, st));
    PROF("row_scale", st, launch_row_scale(n, (int)(w * k), b, 0, (const double*)A, w * lda, P.As, w * k, st));
    rc = tho_two_stage(dtype, n, k0, k, P.Vs, k0w, P.As, k, Q, ldq, R, ldr, S, lds, opts, ws, P.head, stream);
    if (rc) return rc;
    // Q = D^{-1} Q~
    PROF("row_scale", st, launch_row_scale(n, (int)(w * k), b, 1, (const double*)Q, w * ldq, (double*)Q, w * ldq, st));
    return 0;
}

}  // extern "C"
