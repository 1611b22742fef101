// Host-side helpers shared by the entry points of libtho: error reporting,
// optional per-kernel event timing, workspace carving and the chunked
// tall-skinny QR driver (leaf levels, R normalization, formation).
#pragma once

#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/tho.h"
#include "tho_internal.h"

namespace tho {

int set_err(int code, const std::string& msg);
const char* last_error();
int prof_enable(int on);
int prof_collect();
int prof_reset();
int prof_get(int i, char* name, int name_len, double* total_ms, int64_t* launches);

// Address of the calling device's static scratch of tho_two_stage_noalloc
// (set up by its first call on the device; THO_E_UNSUPPORTED before that).
int noalloc_scratch(const void** out);
// Outputs Q, R, S (arguments 9, 11, 13) sharing elements with the inputs
// or each other: -i.  esz = bytes per element.
int check_alias(int64_t n, int64_t k0, int64_t k, int64_t esz, const void* V, int64_t ldv, const void* A,
                int64_t lda, const void* Q, int64_t ldq, const void* R, int64_t ldr, const void* S, int64_t lds);
bool blocks_overlap(const void* p1, int64_t r1, int64_t c1, int64_t ld1, const void* p2, int64_t r2, int64_t c2,
                    int64_t ld2, int64_t esz);

// P and T for the chosen P of §3.2 (k0 x k0 top block, ld k0 outputs) and
// the solves with T^T and T that Algorithm 1 needs (tho_api.cpp).
int p_and_t(int pchoice, int k0, const double* V, int64_t ldv, double* Pm, double* Tm, double* F2, double* pws,
            hipStream_t s);
int solve_tt(int pchoice, int k0, int k, const double* Tm, const double* F2, double* B, int64_t ldb, hipStream_t st);
int solve_t(int pchoice, int k0, int k, const double* Tm, const double* F2, double* B, int64_t ldb, hipStream_t st);
// Householder QR (nonnegative diag R) of an m x k block, k <= 64.
size_t plain_qr_bytes(int64_t m, int64_t k);
int run_plain_qr(int64_t m, int64_t k, const double* X, int64_t ldx, double* Q, int64_t ldq, double* R, int64_t ldr,
                 void* ws, hipStream_t st);

// dtype and size checks shared by the entry points (codes of arguments 1-4).
int check_common(int32_t dtype, int64_t n, int64_t k0, int64_t k);
// Pointer / leading-dimension checks of the (V, A, Q, R, S) argument block
// (codes -5 .. -14 of the tho_two_stage argument order).
int check_io(int64_t k0, int64_t k, const void* V, int64_t ldv, const void* A, int64_t lda, const void* Q,
             int64_t ldq, const void* R, int64_t ldr, const void* S, int64_t lds);

#define HIPCHK(expr)                                                                           \
    do {                                                                                       \
        hipError_t _e = (expr);                                                                \
        if (_e != hipSuccess)                                                                  \
            return ::tho::set_err(THO_E_HIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
    } while (0)

// ---- optional per-kernel timing (benchmark instrumentation)
bool prof_on();
// Returns two events to record around a launch (both null when profiling
// is off) and, after the launch, registers the pair under `name`.
void prof_begin(hipEvent_t* a, hipEvent_t* b);
void prof_end(const char* name, hipEvent_t a, hipEvent_t b);

#define PROF(NAME, st, expr)                                   \
    do {                                                       \
        hipEvent_t _a = nullptr, _b = nullptr;                 \
        if (::tho::prof_on()) ::tho::prof_begin(&_a, &_b);     \
        if (_a) HIPCHK(hipEventRecord(_a, st));                \
        HIPCHK(expr);                                          \
        if (_b) {                                              \
            HIPCHK(hipEventRecord(_b, st));                    \
            ::tho::prof_end(NAME, _a, _b);                     \
        }                                                      \
    } while (0)

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int kp_of(int64_t k) { return k <= 16 ? 16 : (k <= 32 ? 32 : 64); }
inline int k0p_of(int64_t k0) {
    if (k0 == 0) return 0;
    if (k0 <= 16) return 16;
    if (k0 <= 32) return 32;
    if (k0 <= 64) return 64;
    return 128;
}

// Bump allocator over the caller's workspace (256-byte aligned pieces).
// With a null base it only measures.
struct Carve {
    char* base;
    size_t off = 0;
    explicit Carve(void* b) : base((char*)b) {}
    double* take(size_t ndoubles) {
        off = (off + 255) & ~(size_t)255;
        double* p = base ? (double*)(base + off) : nullptr;
        off += ndoubles * sizeof(double);
        return p;
    }
    size_t bytes() const { return off + 256; }
};

hipError_t fill(double* p, int64_t n, double v, hipStream_t st);

// ---- chunked tall-skinny Householder QR of an m x k matrix (k <= 64)
struct LevelPlan {
    int64_t m;
    int nchunk;
    int maxtiles;
};

struct TsqrPlan {
    int64_t m = 0;
    int k = 0, KP = 16;
    std::vector<LevelPlan> lv;
    double *Rtop = nullptr, *G0 = nullptr;
    double* Cfin = nullptr;  // level 0: per chunk KP x KP (two-pass formation)
    std::vector<double*> tau, Tt, stack;  // stack[l] = input matrix of level l (l >= 1)
};

void tsqr_plan(int64_t m, int k, Carve& cv, TsqrPlan& T);

// Level descriptors: level 0 reads X (ld ldx) and writes its Householder
// vectors, later the rows of Q, into Y (ld ldy); Y may equal X.  Level-0
// fields of the fused two-stage path (V, Z, Nc, Nglob) are left empty.
std::vector<TsqrLevel> tsqr_levels(const TsqrPlan& T, const double* X, int64_t ldx, double* Y, int64_t ldy);

// Leaf levels, R with nonnegative diagonal into R (ld ldr), and the
// formation of every level above 0.  k0p is the V width fused into level 0
// (0: none); panel selects the arithmetic of level 0's V products.
int tsqr_factor(const TsqrPlan& T, std::vector<TsqrLevel>& Ls, int k0p, double* R, int64_t ldr, hipStream_t st,
                int panel = 0);
// Formation of level 0 (rows of Q into Ls[0].Y): tsqr_kchain0 (needs the
// formed level 1 only; consumes the level-0 T factors) then tsqr_rows0
// (needs Ls[0].Nglob / Nlp when k0p > 0).  tsqr_form0 runs both in order.
int tsqr_kchain0(const TsqrPlan& T, std::vector<TsqrLevel>& Ls, hipStream_t st);
int tsqr_rows0(const TsqrPlan& T, std::vector<TsqrLevel>& Ls, int k0p, hipStream_t st, int panel = 0);
int tsqr_form0(const TsqrPlan& T, std::vector<TsqrLevel>& Ls, int k0p, hipStream_t st, int panel = 0);

// Split-n reduction out = X^T Y over nrows rows (X: p <= 128 columns, Y:
// q <= 64 columns); `out` is k0p_of(p) x kp_of(q), ld kp_of(q); `part` holds
// xty_plan(nrows).nblk such blocks.
struct XtyPlan {
    int nblk;
    int64_t rows_per_blk;
};
XtyPlan xty_plan(int64_t nrows);
// panel != 0: reduced-precision products (launch_xty_lowp).
int xty(const XtyPlan& xp, int64_t nrows, const double* X, int64_t ldx, int p, const double* Y, int64_t ldy, int q,
        double* part, double* out, hipStream_t st, const char* name, int panel = 0);

// ---- complex path (tho_complex.cpp); k0 <= 64, k <= 32
bool zsupported(int64_t k0, int64_t k);
size_t ztwo_stage_bytes(int64_t n, int64_t k0, int64_t k);
int run_ztwo_stage(int64_t n, int64_t k0, int64_t k, const dcplx* V, int64_t ldv, const dcplx* A, int64_t lda,
                   dcplx* Q, int64_t ldq, dcplx* R, int64_t ldr, dcplx* S, int64_t lds, void* ws, hipStream_t st);
size_t zbcgs_bytes(int64_t n, int64_t k0, int64_t k);
int run_zbcgs(int64_t n, int64_t k0, int64_t k, const dcplx* V, int64_t ldv, const dcplx* A, int64_t lda, dcplx* Q,
              int64_t ldq, dcplx* R, int64_t ldr, dcplx* S, int64_t lds, int proj, int rounds, void* ws,
              hipStream_t st);
size_t zhhqr_bytes(int64_t n, int64_t k0, int64_t k);
size_t ztwo_stage_backward_bytes(int64_t n, int64_t k0, int64_t k);
int run_ztwo_stage_backward(int64_t n, int64_t k0, int64_t k, const dcplx* V, int64_t ldv, const dcplx* A,
                            int64_t lda, const dcplx* Q, int64_t ldq, const dcplx* R, int64_t ldr, const dcplx* gQ,
                            int64_t ldgq, const dcplx* gR, int64_t ldgr, const dcplx* gS, int64_t ldgs, dcplx* dV,
                            int64_t lddv, dcplx* dA, int64_t ldda, void* ws, hipStream_t st);
int run_zhhqr(int64_t n, int64_t k0, int64_t k, const dcplx* V, int64_t ldv, const dcplx* A, int64_t lda, dcplx* Q,
              int64_t ldq, dcplx* R, int64_t ldr, dcplx* S, int64_t lds, void* ws, hipStream_t st);

// Side stream (default priority) and two events per host thread and device:
// the k0 x k0 QR of the top block runs on it beside the first reduction, and
// the level-0 formation chain beside the products that feed the formation.
struct Fork {
    bool ok = false;
    hipStream_t side = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
};
Fork& fork_for_thread();

}  // namespace tho
