// Host helpers of libtho: error state, event timing, the chunked TSQR driver
// and the split-n reduction driver (see tho_host.h).
#include "tho_host.h"

#include <algorithm>

namespace tho {

namespace {
thread_local std::string g_last_error;

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
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

__global__ void k_fill(double* p, int64_t n, double v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
}  // namespace

int set_err(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}
const char* last_error() { return g_last_error.c_str(); }

bool prof_on() { return g_prof_on; }

void prof_begin(hipEvent_t* a, hipEvent_t* b) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    *a = prof_event();
    *b = prof_event();
    if (!*a || !*b) *a = *b = nullptr;
}

void prof_end(const char* name, hipEvent_t a, hipEvent_t b) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_pending.push_back({name, a, b});
}

int prof_enable(int on) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = on != 0;
    return 0;
}

int prof_collect() {
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

int prof_reset() {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_names.clear();
    g_prof_ms.clear();
    g_prof_cnt.clear();
    return 0;
}

int prof_get(int i, char* name, int name_len, double* total_ms, int64_t* launches) {
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

hipError_t fill(double* p, int64_t n, double v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

// Level 0 gets up to 512 chunks (two per compute unit), upper levels one
// tile per chunk (eight wavefronts: four stacked R factors of the level
// below); every chunk has at least k rows so that its first tile can be
// factored on its own.
void tsqr_plan(int64_t m0, int k, Carve& cv, TsqrPlan& T) {
    T.m = m0;
    T.k = k;
    T.KP = kp_of(k);
    T.lv.clear();
    int64_t m = m0;
    for (int level = 0;; level++) {
        const int tb = (level == 0) ? tsqr_tile_rows(T.KP) : tsqr_tile_rows_up(T.KP);
        int64_t nc = cdiv(m, tb);
        if (level == 0) nc = std::min<int64_t>(nc, 512);
        nc = std::max<int64_t>(1, std::min<int64_t>(nc, m / std::max(1, k)));
        const int64_t rows_max = cdiv(m, nc);
        T.lv.push_back({m, (int)nc, (int)cdiv(rows_max, tb)});
        if (nc == 1) break;
        m = nc * k;
    }
    const size_t kk = (size_t)T.KP * T.KP;
    T.Rtop = cv.take(kk);
    T.G0 = cv.take(kk);
    T.Cfin = cv.take((size_t)T.lv[0].nchunk * kk);
    const size_t nl = T.lv.size();
    T.tau.assign(nl, nullptr);
    T.Tt.assign(nl, nullptr);
    T.stack.assign(nl, nullptr);
    for (size_t l = 0; l < nl; l++) {
        const size_t tiles = (size_t)T.lv[l].nchunk * T.lv[l].maxtiles;
        T.tau[l] = cv.take(tiles * T.KP);
        T.Tt[l] = cv.take(tiles * kk);
        if (l >= 1) T.stack[l] = cv.take((size_t)T.lv[l].m * T.KP);
    }
}

std::vector<TsqrLevel> tsqr_levels(const TsqrPlan& T, const double* X, int64_t ldx, double* Y, int64_t ldy) {
    const int nl = (int)T.lv.size();
    std::vector<TsqrLevel> Ls(nl);
    for (int l = 0; l < nl; l++) {
        TsqrLevel& L = Ls[l];
        std::memset(&L, 0, sizeof(L));
        L.m = T.lv[l].m;
        L.k = T.k;
        L.nchunk = T.lv[l].nchunk;
        L.maxtiles = T.lv[l].maxtiles;
        if (l == 0) {
            L.X = X;
            L.ldx = ldx;
            L.Y = Y;
            L.ldy = ldy;
        } else {
            L.X = T.stack[l];
            L.ldx = T.KP;
            L.Y = T.stack[l];
            L.ldy = T.KP;
        }
        L.tau = T.tau[l];
        L.Tt = T.Tt[l];
        L.Cfin = (l == 0) ? T.Cfin : nullptr;
        L.Rnext = (l + 1 < nl) ? T.stack[l + 1] : T.Rtop;
        L.ldrn = T.KP;
        if (l + 1 < nl) {
            L.Gin = T.stack[l + 1];
            L.ldg = T.KP;
            L.gstride = T.k;
        } else {
            L.Gin = T.G0;
            L.ldg = T.KP;
            L.gstride = 0;
        }
    }
    return Ls;
}

int tsqr_factor(const TsqrPlan& T, std::vector<TsqrLevel>& Ls, int k0p, double* R, int64_t ldr, hipStream_t st,
                int panel) {
    const int nl = (int)Ls.size();
    for (int l = 0; l < nl; l++)
        PROF(l == 0 ? "leaf_l0" : "leaf_up", st,
             l == 0 ? launch_tsqr_leaf(T.KP, k0p, panel, Ls[l], st) : launch_tsqr_leaf_up(T.KP, Ls[l], st));
    // R with nonnegative diagonal; the top-level Q starts from the sign matrix
    PROF("finish_r", st, launch_finish_r(T.k, T.KP, T.Rtop, T.KP, R, ldr, T.G0, st));
    for (int l = nl - 1; l >= 1; l--) PROF("form_up", st, launch_tsqr_form_up(T.KP, Ls[l], st));
    return 0;
}

int tsqr_kchain0(const TsqrPlan& T, std::vector<TsqrLevel>& Ls, hipStream_t st) {
    PROF("kchain_l0", st, launch_tsqr_kchain(T.KP, Ls[0], st));
    return 0;
}

int tsqr_rows0(const TsqrPlan& T, std::vector<TsqrLevel>& Ls, int k0p, hipStream_t st, int panel) {
    PROF("form_l0", st, launch_tsqr_rows(T.KP, k0p, panel, Ls[0], st));
    return 0;
}

int tsqr_form0(const TsqrPlan& T, std::vector<TsqrLevel>& Ls, int k0p, hipStream_t st, int panel) {
    int rc = tsqr_kchain0(T, Ls, st);
    if (rc) return rc;
    return tsqr_rows0(T, Ls, k0p, st, panel);
}

// two workgroups per compute unit, >= 64 rows each (all resident at once,
// with room left beside them for the one-workgroup QR of the top block)
XtyPlan xty_plan(int64_t nrows) {
    XtyPlan xp;
    int64_t nb = std::max<int64_t>(1, std::min<int64_t>(512, cdiv(nrows, 64)));
    xp.rows_per_blk = std::max<int64_t>(16, cdiv(cdiv(nrows, nb), 16) * 16);
    xp.nblk = (int)std::max<int64_t>(1, cdiv(nrows, xp.rows_per_blk));
    return xp;
}

int xty(const XtyPlan& xp, int64_t nrows, const double* X, int64_t ldx, int p, const double* Y, int64_t ldy, int q,
        double* part, double* out, hipStream_t st, const char* name, int panel) {
    const int pp = k0p_of(p), qp = kp_of(q);
    if (pp == 0) return 0;
    if (panel != 0)
        PROF(name, st, launch_xty_lowp(panel, pp / 16, qp / 16, nrows, X, ldx, p, Y, ldy, q, xp.nblk, xp.rows_per_blk,
                                       part, st));
    else
        PROF(name, st, launch_xty_partial(pp / 16, qp / 16, nrows, X, ldx, p, Y, ldy, q, xp.nblk, xp.rows_per_blk,
                                          part, st));
    PROF("reduce_parts", st, launch_reduce_parts(xp.nblk, (int64_t)pp * qp, part, out, st));
    return 0;
}

Fork& fork_for_thread() {
    thread_local std::vector<Fork> forks;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    if ((int)forks.size() <= dev) forks.resize(dev + 1);
    Fork& f = forks[dev];
    if (!f.ok) {
        f.ok = hipStreamCreateWithFlags(&f.side, hipStreamNonBlocking) == hipSuccess &&
               hipEventCreateWithFlags(&f.ev0, hipEventDisableTiming) == hipSuccess &&
               hipEventCreateWithFlags(&f.ev1, hipEventDisableTiming) == hipSuccess;
    }
    return f;
}

}  // namespace tho
