// C ABI of libtho: argument validation, workspace layout and the launch
// sequence of the two-stage Householder orthogonalization (Algorithm 1 of
// He & Shao, second choice of P) on one HIP stream.  No host
// synchronization and no device allocation happen here.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>
#include <mutex>

#include "../../include/tho.h"
#include "tho_internal.h"

using namespace tho;

namespace {

thread_local std::string g_last_error;

int set_err(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

#define HIPCHK(expr)                                                                      \
    do {                                                                                  \
        hipError_t _e = (expr);                                                           \
        if (_e != hipSuccess)                                                             \
            return set_err(THO_E_HIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
    } while (0)

// ---- optional per-kernel timing (benchmark instrumentation)
struct ProfRec {
    const char* name;
    hipEvent_t a, b;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof_pending;
std::vector<hipEvent_t> g_prof_pool;
std::vector<std::string> g_prof_names;
std::vector<double> g_prof_ms;
std::vector<int64_t> g_prof_cnt;

hipEvent_t prof_event() {
    if (!g_prof_pool.empty()) {
        hipEvent_t e = g_prof_pool.back();
        g_prof_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    hipEventCreate(&e);
    return e;
}

// Records an event pair around `expr` on stream `st` when profiling is on.
#define PROF(NAME, st, expr)                                             \
    do {                                                                 \
        hipEvent_t _a = nullptr, _b = nullptr;                           \
        if (g_prof_on) {                                                 \
            std::lock_guard<std::mutex> _lk(g_prof_mu);                  \
            _a = prof_event();                                           \
            _b = prof_event();                                           \
        }                                                                \
        if (_a) HIPCHK(hipEventRecord(_a, st));                          \
        HIPCHK(expr);                                                    \
        if (_b) {                                                        \
            HIPCHK(hipEventRecord(_b, st));                              \
            std::lock_guard<std::mutex> _lk(g_prof_mu);                  \
            g_prof_pending.push_back({NAME, _a, _b});                    \
        }                                                                \
    } while (0)

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int pad16(int64_t x) { return (int)(cdiv(x, 16) * 16); }

int kp_of(int64_t k) { return k <= 16 ? 16 : (k <= 32 ? 32 : 64); }
int k0p_of(int64_t k0) {
    if (k0 == 0) return 0;
    if (k0 <= 16) return 16;
    if (k0 <= 32) return 32;
    if (k0 <= 64) return 64;
    return 128;
}
int mt_of(int k0p) { return k0p / 16; }

// Bump allocator over the caller's workspace (256-byte aligned pieces).
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
};

struct LevelPlan {
    int64_t m;
    int nchunk;
    int maxtiles;
};

// Chunking of the chunked tall-skinny QR: level 0 gets up to 512 chunks
// (two per compute unit), upper levels one tile per chunk; every chunk has
// at least k rows so its first tile can be factored on its own.
std::vector<LevelPlan> plan_levels(int64_t m0, int k, int kp) {
    std::vector<LevelPlan> lv;
    const int tb = tsqr_tile_rows(kp);
    int64_t m = m0;
    for (int level = 0;; level++) {
        int64_t nc = cdiv(m, tb);
        if (level == 0) nc = std::min<int64_t>(nc, 512);
        nc = std::max<int64_t>(1, std::min<int64_t>(nc, m / std::max(1, k)));
        const int64_t rows_max = cdiv(m, nc);
        lv.push_back({m, (int)nc, (int)cdiv(rows_max, tb)});
        if (nc == 1) break;
        m = nc * k;
    }
    return lv;
}

struct TwoStagePlan {
    int KP, K0P;
    int nblk1;  // phase-1 reduction blocks
    int64_t rows_per_blk1;
    std::vector<LevelPlan> lv;
    // workspace pieces
    double *part, *Cbuf, *Pm, *Tm, *Zbuf, *A1top, *Mbuf, *Nglob, *Rtop, *G0, *Nc, *prod, *Zperm, *Nperm;
    std::vector<double*> tau, Tt, stack;  // stack[l] = input matrix of level l (l >= 1)
    size_t bytes;
};

void make_plan(int64_t n, int64_t k0, int64_t k, void* ws, TwoStagePlan& P) {
    P.KP = kp_of(k);
    P.K0P = k0p_of(k0);
    const int64_t m0 = n - k0;
    P.lv = plan_levels(m0, (int)k, P.KP);
    // phase 1: about 4 workgroups per compute unit, >= 64 rows each
    P.nblk1 = (int)std::max<int64_t>(1, std::min<int64_t>(1024, cdiv(n, 64)));
    P.rows_per_blk1 = cdiv(cdiv(n, P.nblk1), 16) * 16;
    P.nblk1 = (int)cdiv(n, P.rows_per_blk1);
    Carve cv(ws);
    const size_t kk = (size_t)P.KP * P.KP;
    const size_t nk = (size_t)std::max(P.K0P, 16) * P.KP;
    const int nc0 = P.lv[0].nchunk;
    if (k0 > 0) {
        P.part = cv.take((size_t)std::max(P.nblk1, nc0) * nk);
        P.Cbuf = cv.take(nk);
        P.Pm = cv.take((size_t)k0 * k0);
        P.Tm = cv.take((size_t)k0 * k0);
        P.Zbuf = cv.take(nk);
        P.A1top = cv.take((size_t)k0 * P.KP);
        P.Mbuf = cv.take(nk);
        P.Nglob = cv.take(nk);
        P.Nc = cv.take((size_t)nc0 * nk);
        P.Zperm = cv.take(nk);
        P.Nperm = cv.take(nk);
        P.prod = P.part;
    } else {
        P.part = P.Cbuf = P.Pm = P.Tm = P.Zbuf = P.A1top = P.Mbuf = P.Nglob = P.Nc = P.prod = nullptr;
        P.Zperm = P.Nperm = nullptr;
    }
    P.Rtop = cv.take(kk);
    P.G0 = cv.take(kk);
    P.tau.assign(P.lv.size(), nullptr);
    P.Tt.assign(P.lv.size(), nullptr);
    P.stack.assign(P.lv.size(), nullptr);
    for (size_t l = 0; l < P.lv.size(); l++) {
        const size_t tiles = (size_t)P.lv[l].nchunk * P.lv[l].maxtiles;
        P.tau[l] = cv.take(tiles * P.KP);
        P.Tt[l] = cv.take(tiles * kk);
        if (l >= 1) P.stack[l] = cv.take((size_t)P.lv[l].m * P.KP);
    }
    P.bytes = cv.off + 256;
}

__global__ void k_fill(double* p, int64_t n, double v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

hipError_t fill(double* p, int64_t n, double v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

#ifdef THO_DEBUG_SPLIT_VN
__global__ void k_dbg_add_vn(int64_t m, int k, int k0, const double* V, int64_t ldv, const double* N, int ldn,
                             double* Q, int64_t ldq) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m * k) return;
    const int64_t i = e / k; const int j = (int)(e % k);
    double s = 0.0;
    for (int p = 0; p < k0; p++) s += V[i * ldv + p] * N[p * ldn + j];
    Q[i * ldq + j] += s;
}
#endif

int check_common(int32_t dtype, int64_t n, int64_t k0, int64_t k) {
    if (dtype != THO_F64 && dtype != THO_C128) return set_err(-1, "dtype must be THO_F64 or THO_C128");
    if (n < 0) return set_err(-2, "n must be >= 0");
    if (k0 < 0 || k0 > THO_MAX_K0) return set_err(-3, "k0 out of range [0, THO_MAX_K0]");
    if (k < 0 || k > THO_MAX_K) return set_err(-4, "k out of range [0, THO_MAX_K]");
    if (n < k0 + k) return set_err(-2, "need n >= k0 + k");
    return 0;
}

}  // namespace

#ifdef THO_DEBUG_SKIP_FORM0
static size_t g_dbg_tt_off = 0, g_dbg_nc_off = 0, g_dbg_st1_off = 0, g_dbg_ng_off = 0;
extern "C" size_t tho_debug_nglob(void) { return g_dbg_ng_off; }
static int64_t g_dbg_m1 = 0;
static int g_dbg_maxtiles = 0, g_dbg_nchunk = 0;
extern "C" void tho_debug_offsets(size_t* tt, size_t* nc, int* maxtiles, int* nchunk) {
    *tt = g_dbg_tt_off; *nc = g_dbg_nc_off; *maxtiles = g_dbg_maxtiles; *nchunk = g_dbg_nchunk;
}
extern "C" void tho_debug_stack1(size_t* off, int64_t* m1) { *off = g_dbg_st1_off; *m1 = g_dbg_m1; }
#endif

extern "C" {

const char* tho_version(void) { return "tho 0.1.0 (gfx950)"; }

const char* tho_last_error(void) { return g_last_error.c_str(); }

const char* tho_strerror(int code) {
    if (code == 0) return "success";
    if (code == THO_E_WORKSPACE) return "workspace too small";
    if (code == THO_E_HIP) return "HIP runtime error";
    if (code == THO_E_UNSUPPORTED) return "unsupported combination of arguments";
    if (code < 0) return "invalid argument";
    return "unknown code";
}

int tho_profile_enable(int on) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = on != 0;
    return 0;
}

int tho_profile_collect(void) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (auto& r : g_prof_pending) {
        hipError_t e = hipEventSynchronize(r.b);
        if (e != hipSuccess) return set_err(THO_E_HIP, std::string("hipEventSynchronize: ") + hipGetErrorString(e));
        float ms = 0.f;
        hipEventElapsedTime(&ms, r.a, r.b);
        size_t i = 0;
        while (i < g_prof_names.size() && g_prof_names[i] != r.name) i++;
        if (i == g_prof_names.size()) {
            g_prof_names.push_back(r.name);
            g_prof_ms.push_back(0.0);
            g_prof_cnt.push_back(0);
        }
        g_prof_ms[i] += ms;
        g_prof_cnt[i] += 1;
        g_prof_pool.push_back(r.a);
        g_prof_pool.push_back(r.b);
    }
    g_prof_pending.clear();
    return (int)g_prof_names.size();
}

int tho_profile_reset(void) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_names.clear();
    g_prof_ms.clear();
    g_prof_cnt.clear();
    return 0;
}

int tho_profile_get(int i, char* name, int name_len, double* total_ms, int64_t* launches) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (i < 0 || i >= (int)g_prof_names.size()) return set_err(-1, "profile index out of range");
    if (name && name_len > 0) {
        std::strncpy(name, g_prof_names[i].c_str(), (size_t)name_len - 1);
        name[name_len - 1] = 0;
    }
    if (total_ms) *total_ms = g_prof_ms[i];
    if (launches) *launches = g_prof_cnt[i];
    return 0;
}

int tho_two_stage_workspace(int32_t dtype, int64_t n, int64_t k0, int64_t k, const tho_opts_t* opts,
                            size_t* bytes) {
    int rc = check_common(dtype, n, k0, k);
    if (rc) return rc;
    if (!bytes) return set_err(-6, "bytes must not be NULL");
    (void)opts;
    if (k == 0) { *bytes = 0; return 0; }
    TwoStagePlan P;
    make_plan(n, k0, k, nullptr, P);
    *bytes = P.bytes;
    return 0;
}

int tho_two_stage(int32_t dtype, int64_t n, int64_t k0, int64_t k, const void* V_, int64_t ldv,
                  const void* A_, int64_t lda, void* Q_, int64_t ldq, void* R_, int64_t ldr, void* S_,
                  int64_t lds, const tho_opts_t* opts, void* ws, size_t ws_bytes, void* stream) {
    int rc = check_common(dtype, n, k0, k);
    if (rc) return rc;
    if (dtype != THO_F64) return set_err(THO_E_UNSUPPORTED, "only THO_F64 is implemented");
    if (opts && (opts->p_choice != THO_P_QR || opts->panel != THO_PANEL_F64 || opts->flags != 0))
        return set_err(THO_E_UNSUPPORTED, "only p_choice=THO_P_QR, panel=THO_PANEL_F64 are implemented");
    if (k == 0) return 0;
    if (k0 > 0 && !V_) return set_err(-5, "V is NULL");
    if (k0 > 0 && ldv < k0) return set_err(-6, "ldv < k0");
    if (!A_) return set_err(-7, "A is NULL");
    if (lda < k) return set_err(-8, "lda < k");
    if (!Q_) return set_err(-9, "Q is NULL");
    if (ldq < k) return set_err(-10, "ldq < k");
    if (!R_) return set_err(-11, "R is NULL");
    if (ldr < k) return set_err(-12, "ldr < k");
    if (k0 > 0 && !S_) return set_err(-13, "S is NULL");
    if (k0 > 0 && lds < k) return set_err(-14, "lds < k");
    for (const void* p : {V_, A_, (const void*)Q_, (const void*)R_, (const void*)S_})
        if (p && ((uintptr_t)p & 7)) return set_err(-5, "matrices must be 8-byte aligned");
    if (!ws) return set_err(-16, "workspace is NULL");
    TwoStagePlan P;
    make_plan(n, k0, k, nullptr, P);
    if (ws_bytes < P.bytes) return set_err(THO_E_WORKSPACE, "workspace too small");
    make_plan(n, k0, k, ws, P);

    hipStream_t st = (hipStream_t)stream;
    const double* V = (const double*)V_;
    const double* A = (const double*)A_;
    double* Q = (double*)Q_;
    double* R = (double*)R_;
    double* S = (double*)S_;
    const int KP = P.KP, K0P = P.K0P;
    const int ik = (int)k, ik0 = (int)k0;
    const size_t nk = (size_t)std::max(K0P, 16) * KP;

    if (k0 > 0) {
        // line 1, second choice: V_top = Q1 R1, P = -Q1, T = I + R1^T
        PROF("qr_top", st, launch_qr_top(ik0, V, ldv, P.Pm, P.Tm, st));
        // line 4 reduction: C = V^T A over all n rows
        PROF("xty_partial", st, launch_xty_partial(mt_of(K0P), KP / 16, n, V, ldv, ik0, A, lda, ik, P.nblk1,
                                  P.rows_per_blk1, P.part, st));
        PROF("reduce_parts", st, launch_reduce_parts(P.nblk1, (int64_t)K0P * KP, P.part, P.Cbuf, st));
        // W^T A = P^T A_top - C ;  Z = T^{-T} (W^T A)
        PROF("fill", st, fill(P.Zbuf, (int64_t)nk, 0.0, st));
        PROF("small_gemm", st, launch_small_gemm(ik0, ik, ik0, 1.0, P.Pm, k0, 1, A, lda, 0, -1.0, P.Cbuf, KP, P.Zbuf,
                                 KP, st));
        PROF("trsm", st, launch_trsm_lower(ik0, ik, P.Tm, k0, 1, P.Zbuf, KP, st));
        PROF("permute", st, launch_permute_b(K0P, KP, P.Zbuf, P.Zperm, st));
        // A1_top = A_top - (P - V_top) Z ;  S = P^T A1_top  (line 5)
        PROF("small_gemm", st, launch_small_gemm(ik0, ik, ik0, -1.0, P.Pm, k0, 0, P.Zbuf, KP, 0, 1.0, A, lda, P.A1top,
                                 KP, st));
        PROF("small_gemm", st, launch_small_gemm(ik0, ik, ik0, 1.0, V, ldv, 0, P.Zbuf, KP, 0, 1.0, P.A1top, KP,
                                 P.A1top, KP, st));
        PROF("small_gemm", st, launch_small_gemm(ik0, ik, ik0, 1.0, P.Pm, k0, 1, P.A1top, KP, 0, 0.0, nullptr, 0, S,
                                 lds, st));
    }

    // line 6: chunked Householder QR of A_low (+ V Z on the fly)
    const int nl = (int)P.lv.size();
    std::vector<TsqrLevel> Ls(nl);
    for (int l = 0; l < nl; l++) {
        TsqrLevel& L = Ls[l];
        std::memset(&L, 0, sizeof(L));
        L.m = P.lv[l].m;
        L.k = ik;
        L.nchunk = P.lv[l].nchunk;
        L.maxtiles = P.lv[l].maxtiles;
        if (l == 0) {
            L.X = A + k0 * lda;
            L.ldx = lda;
            L.Y = Q + k0 * ldq;
            L.ldy = ldq;
            if (k0 > 0) {
                L.V = V + k0 * ldv;
                L.ldv = ldv;
                L.k0 = ik0;
                L.Z = P.Zperm;
                L.Nc = P.Nc;
                L.Nglob = P.Nperm;
            }
        } else {
            L.X = P.stack[l];
            L.ldx = KP;
            L.Y = P.stack[l];
            L.ldy = KP;
        }
        L.tau = P.tau[l];
        L.Tt = P.Tt[l];
        L.Rnext = (l + 1 < nl) ? P.stack[l + 1] : P.Rtop;
        L.ldrn = KP;
        if (l + 1 < nl) {
            L.Gin = P.stack[l + 1];
            L.ldg = KP;
            L.gstride = ik;
        } else {
            L.Gin = P.G0;
            L.ldg = KP;
            L.gstride = 0;
        }
    }
    for (int l = 0; l < nl; l++)
        PROF(l == 0 ? "leaf_l0" : "leaf_up", st, launch_tsqr_leaf(KP, l == 0 ? K0P : 0, Ls[l], st));
    // R with nonnegative diagonal; the top-level Q starts from the sign matrix
    PROF("finish_r", st, launch_finish_r(ik, KP, P.Rtop, KP, R, ldr, P.G0, st));
    for (int l = nl - 1; l >= 1; l--) PROF("form_up", st, launch_tsqr_form(KP, 0, Ls[l], st));

    if (k0 > 0) {
        // line 7: G = W^T [0; Q_] = -sum_c N_c G_c ;  N = T^{-1} G
        PROF("chunk_prod", st, launch_chunk_prod(Ls[0].nchunk, K0P, KP, ik, P.Nc, Ls[0].Gin, Ls[0].ldg, Ls[0].gstride,
                                 P.prod, st));
        PROF("reduce_parts", st, launch_reduce_parts(Ls[0].nchunk, (int64_t)K0P * KP, P.prod, P.Mbuf, st));
        PROF("small_gemm", st, launch_small_gemm(K0P, KP, 0, 0.0, P.Mbuf, KP, 0, P.Mbuf, KP, 0, -1.0, P.Mbuf, KP,
                                 P.Nglob, KP, st));
        PROF("trsm", st, launch_trsm_lower(ik0, ik, P.Tm, k0, 0, P.Nglob, KP, st));
        PROF("permute", st, launch_permute_b(K0P, KP, P.Nglob, P.Nperm, st));
        // Q_top = -(P - V_top) N
        PROF("small_gemm", st, launch_small_gemm(ik0, ik, ik0, 1.0, V, ldv, 0, P.Nglob, KP, 0, 0.0, nullptr, 0, Q, ldq,
                                 st));
        PROF("small_gemm", st, launch_small_gemm(ik0, ik, ik0, -1.0, P.Pm, k0, 0, P.Nglob, KP, 0, 1.0, Q, ldq, Q, ldq,
                                 st));
    }
#ifdef THO_DEBUG_SKIP_FORM0
    g_dbg_st1_off = (nl > 1) ? (size_t)((char*)P.stack[1] - (char*)ws) : 0;
    g_dbg_ng_off = P.Nglob ? (size_t)((char*)P.Nglob - (char*)ws) : 0;
    g_dbg_m1 = (nl > 1) ? P.lv[1].m : 0;
    g_dbg_tt_off = (size_t)((char*)P.Tt[0] - (char*)ws);
    g_dbg_nc_off = P.Nc ? (size_t)((char*)P.Nc - (char*)ws) : 0;
    g_dbg_maxtiles = P.lv[0].maxtiles;
    g_dbg_nchunk = P.lv[0].nchunk;
    return 0;
#endif
#ifdef THO_DEBUG_SPLIT_VN
    if (k0 > 0) {
        PROF("form_l0", st, launch_tsqr_form(KP, 0, Ls[0], st));
        hipLaunchKernelGGL(k_dbg_add_vn, dim3((unsigned)cdiv((n - k0) * k, 256)), dim3(256), 0, st,
                           n - k0, ik, ik0, V + k0 * ldv, ldv, (const double*)P.Nglob, KP, Q + k0 * ldq, ldq);
        return 0;
    }
#endif
    PROF("form_l0", st, launch_tsqr_form(KP, K0P, Ls[0], st));
    return 0;
}

}  // extern "C"
