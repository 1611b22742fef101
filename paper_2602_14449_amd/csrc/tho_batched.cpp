// Batched entry points: many independent two-stage problems in one
// persistent launch (k_batched.hip), captured once into a HIP graph.
//
// Plan creation validates the problems, lays out each problem's workspace,
// orders the problems longest first, picks the tile height (128 or 256 rows)
// and the number of persistent workgroups by timing the candidates on the
// actual batch (the choice is cached per batch signature and device for the
// process, and in the file THO_TUNE_CACHE names, if set),
// and captures the launch sequence (counter reset + one persistent kernel per
// column-width class) into a graph that tho_batched_run replays.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <tuple>

#include "tho_host.h"

using namespace tho;

struct tho_plan_s {
    static constexpr int MAXG = 12;  // (column class, V width class) groups
    static constexpr int NSTREAM = 4;
    int count = 0;
    int ngroups = 0;
    int kp[MAXG] = {}, k0p[MAXG] = {}, gcount[MAXG] = {}, goff[MAXG] = {};
    BatchedInst* d_inst = nullptr;
    TsqrLevel* d_lv = nullptr;
    int* d_order = nullptr;
    int* d_counter = nullptr;
    int rbo = 4, grid = 0;
    double tuned_ms = 0.0;
    hipStream_t cs = nullptr;
    hipStream_t fork[NSTREAM] = {};
    hipEvent_t ev[NSTREAM + 1] = {};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

constexpr int MIN_TILE = 128;  // smallest candidate tile height

// Autotuner results: process-global, and shared across processes through a
// text file when the environment variable THO_TUNE_CACHE names one.  A line
// of the file is
//     tho-batched-v1 <arch> <compute units> <count> <sum n> <sum k0> <sum k> <tile blocks> <grid>
// (the batch signature, the device it was measured on, the choice); lines
// that do not parse or belong to another device are ignored.
using TuneKey = std::tuple<std::string, int, int, int64_t, int64_t, int64_t>;
std::mutex g_tune_mu;
std::map<TuneKey, std::pair<int, int>> g_tune_cache;
bool g_tune_file_read = false;

const char* tune_file() {
    const char* f = std::getenv("THO_TUNE_CACHE");
    return (f && *f) ? f : nullptr;
}

// Under g_tune_mu.
void tune_file_load() {
    if (g_tune_file_read) return;
    g_tune_file_read = true;
    const char* path = tune_file();
    if (!path) return;
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    char line[512], arch[128];
    while (std::fgets(line, sizeof line, f)) {
        int cus = 0, count = 0, rbo = 0, grid = 0;
        long long sn = 0, sk0 = 0, sk = 0;
        if (std::sscanf(line, "tho-batched-v1 %127s %d %d %lld %lld %lld %d %d", arch, &cus, &count, &sn, &sk0, &sk,
                        &rbo, &grid) == 8 &&
            (rbo == 2 || rbo == 4) && grid > 0)
            g_tune_cache[TuneKey(arch, cus, count, sn, sk0, sk)] = {rbo, grid};
    }
    std::fclose(f);
}

// Under g_tune_mu; best effort (a cache that cannot be written is not an error).
void tune_file_append(const TuneKey& k, int rbo, int grid) {
    const char* path = tune_file();
    if (!path) return;
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "tho-batched-v1 %s %d %d %lld %lld %lld %d %d\n", std::get<0>(k).c_str(), std::get<1>(k),
                 std::get<2>(k), (long long)std::get<3>(k), (long long)std::get<4>(k), (long long)std::get<5>(k), rbo,
                 grid);
    std::fclose(f);
}

size_t inst_doubles(int64_t n, int64_t k0, int64_t k) {
    const int KP = kp_of(k), K0P = k0p_of(k0);
    const int64_t tiles = cdiv(n - k0, MIN_TILE);
    // Pm, Tm, Zperm, Nperm, Nc, Rtop, G0, tau, Tt (+ 256-byte alignment slack)
    return (size_t)(2 * k0 * k0 + 3 * (int64_t)K0P * KP + 2 * KP * KP + tiles * KP + tiles * KP * KP) + 9 * 32;
}

int check_problems(int32_t count, const tho_problem_t* probs) {
    if (count < 0) return set_err(-1, "count must be >= 0");
    if (count > 0 && !probs) return set_err(-2, "problems is NULL");
    for (int i = 0; i < count; i++) {
        const tho_problem_t& p = probs[i];
        const std::string at = " (problem " + std::to_string(i) + ")";
        if (p.k0 < 0 || p.k0 > THO_BATCHED_MAX_K0) return set_err(-2, "k0 out of range [0, THO_BATCHED_MAX_K0]" + at);
        if (p.k < 0 || p.k > THO_MAX_K) return set_err(-2, "k out of range [0, THO_MAX_K]" + at);
        if (p.n < p.k0 + p.k) return set_err(-2, "need n >= k0 + k" + at);
        if (p.k == 0) continue;
        if (p.k0 > 0 && (!p.V || p.ldv < p.k0)) return set_err(-2, "bad V or ldv" + at);
        if (!p.A || p.lda < p.k) return set_err(-2, "bad A or lda" + at);
        if (!p.Q || p.ldq < p.k) return set_err(-2, "bad Q or ldq" + at);
        if (!p.R || p.ldr < p.k) return set_err(-2, "bad R or ldr" + at);
        if (p.k0 > 0 && (!p.S || p.lds < p.k)) return set_err(-2, "bad S or lds" + at);
        for (const void* q : {p.V, p.A, (const void*)p.Q, (const void*)p.R, (const void*)p.S})
            if (q && ((uintptr_t)q & 7)) return set_err(-2, "matrices must be 8-byte aligned" + at);
    }
    return 0;
}

size_t batched_bytes(int32_t count, const tho_problem_t* probs) {
    Carve cv(nullptr);
    for (int i = 0; i < count; i++)
        if (probs[i].k > 0) cv.take(inst_doubles(probs[i].n, probs[i].k0, probs[i].k));
    return cv.bytes();
}

// Counter reset on `st`, then the groups spread over the fork streams (so
// that the tail of one group overlaps the others), joined back into `st`.
int launch_all(tho_plan_s* P, int rbo, int grid, hipStream_t st) {
    HIPCHK(launch_zero_ints(P->d_counter, P->ngroups, st));
    const int ns = std::min(P->ngroups, (int)tho_plan_s::NSTREAM);
    HIPCHK(hipEventRecord(P->ev[0], st));
    for (int s = 0; s < ns; s++) HIPCHK(hipStreamWaitEvent(P->fork[s], P->ev[0], 0));
    for (int gi = 0; gi < P->ngroups; gi++) {
        const int r = (P->kp[gi] >= 64) ? 2 : rbo;
        HIPCHK(launch_batched(P->kp[gi], P->k0p[gi], r, P->d_inst, P->d_lv, P->d_order + P->goff[gi], P->gcount[gi],
                              P->d_counter + gi, grid, P->fork[gi % ns]));
    }
    for (int s = 0; s < ns; s++) {
        HIPCHK(hipEventRecord(P->ev[s + 1], P->fork[s]));
        HIPCHK(hipStreamWaitEvent(st, P->ev[s + 1], 0));
    }
    return 0;
}

void destroy(tho_plan_s* P) {
    if (!P) return;
    if (P->exec) hipGraphExecDestroy(P->exec);
    if (P->graph) hipGraphDestroy(P->graph);
    if (P->cs) hipStreamDestroy(P->cs);
    for (auto& f : P->fork)
        if (f) hipStreamDestroy(f);
    for (auto& e : P->ev)
        if (e) hipEventDestroy(e);
    if (P->d_inst) hipFree(P->d_inst);
    if (P->d_lv) hipFree(P->d_lv);
    if (P->d_order) hipFree(P->d_order);
    if (P->d_counter) hipFree(P->d_counter);
    delete P;
}

}  // namespace

extern "C" {

int tho_batched_workspace(int32_t count, const tho_problem_t* probs, const tho_opts_t* opts, size_t* bytes) {
    int rc = check_problems(count, probs);
    if (rc) return rc;
    if (opts && (opts->panel != THO_PANEL_F64 || opts->flags != 0 || opts->p_choice != THO_P_QR))
        return set_err(THO_E_UNSUPPORTED, "the batched path supports the default options only");
    if (!bytes) return set_err(-4, "bytes must not be NULL");
    *bytes = batched_bytes(count, probs);
    return 0;
}

int tho_batched_plan_create(int32_t count, const tho_problem_t* probs, void* ws, size_t ws_bytes,
                            const tho_opts_t* opts, void* stream, tho_plan_t* plan) {
    int rc = check_problems(count, probs);
    if (rc) return rc;
    if (opts && (opts->panel != THO_PANEL_F64 || opts->flags != 0 || opts->p_choice != THO_P_QR))
        return set_err(THO_E_UNSUPPORTED, "the batched path supports the default options only");
    if (!plan) return set_err(-7, "plan must not be NULL");
    *plan = nullptr;
    if (ws_bytes < batched_bytes(count, probs)) return set_err(THO_E_WORKSPACE, "workspace too small");
    if (!ws && count > 0) return set_err(-3, "workspace is NULL");

    tho_plan_s* P = new tho_plan_s();
    std::vector<BatchedInst> inst;
    std::vector<TsqrLevel> lv;
    std::vector<int> idx;
    Carve cv(ws);
    int64_t sig_n = 0, sig_k0 = 0, sig_k = 0;
    for (int i = 0; i < count; i++) {
        const tho_problem_t& p = probs[i];
        if (p.k == 0) continue;
        const int KP = kp_of(p.k), K0P = k0p_of(p.k0);
        const int64_t m = p.n - p.k0;
        const int maxtiles = (int)cdiv(m, MIN_TILE);
        BatchedInst b{};
        b.n = p.n;
        b.k0 = (int)p.k0;
        b.k = (int)p.k;
        b.K0P = K0P;
        b.V = (const double*)p.V;
        b.A = (const double*)p.A;
        b.Q = (double*)p.Q;
        b.R = (double*)p.R;
        b.S = (double*)p.S;
        b.ldv = p.ldv;
        b.lda = p.lda;
        b.ldq = p.ldq;
        b.ldr = p.ldr;
        b.lds = p.lds;
        b.Pm = cv.take((size_t)p.k0 * p.k0);
        b.Tm = cv.take((size_t)p.k0 * p.k0);
        b.Zperm = cv.take((size_t)K0P * KP);
        b.Nperm = cv.take((size_t)K0P * KP);
        b.Nc = cv.take((size_t)K0P * KP);
        b.Rtop = cv.take((size_t)KP * KP);
        b.G0 = cv.take((size_t)KP * KP);
        TsqrLevel L;
        std::memset(&L, 0, sizeof(L));
        L.m = m;
        L.k = (int)p.k;
        L.nchunk = 1;
        L.maxtiles = maxtiles;
        L.X = b.A + p.k0 * p.lda;
        L.ldx = p.lda;
        L.Y = b.Q + p.k0 * p.ldq;
        L.ldy = p.ldq;
        if (p.k0 > 0) {
            L.V = b.V + p.k0 * p.ldv;
            L.ldv = p.ldv;
            L.k0 = (int)p.k0;
            L.Z = b.Zperm;
            L.Nc = b.Nc;
            L.Nglob = b.Nperm;
        }
        L.tau = cv.take((size_t)maxtiles * KP);
        L.Tt = cv.take((size_t)maxtiles * KP * KP);
        L.Rnext = b.Rtop;
        L.ldrn = KP;
        L.Gin = b.G0;
        L.ldg = KP;
        L.gstride = 0;
        inst.push_back(b);
        lv.push_back(L);
        idx.push_back((int)inst.size() - 1);
        sig_n += p.n;
        sig_k0 += p.k0;
        sig_k += p.k;
    }
    P->count = (int)inst.size();
    // groups by (column class, V width class), longest problems first inside
    // each group; groups with more work are launched first
    auto work = [&](int i) { return inst[i].n * (int64_t)(inst[i].k0 + 2 * inst[i].k); };
    std::vector<std::pair<int64_t, std::vector<int>>> groups;
    std::vector<std::pair<int, int>> gkey;
    for (int kp : {16, 32, 64})
        for (int k0p : {0, 16, 32, 64}) {
            std::vector<int> g;
            int64_t wsum = 0;
            for (int i : idx)
                if (kp_of(inst[i].k) == kp && inst[i].K0P == k0p) {
                    g.push_back(i);
                    wsum += work(i);
                }
            if (g.empty()) continue;
            std::stable_sort(g.begin(), g.end(), [&](int a, int b) { return work(a) > work(b); });
            groups.push_back({wsum, g});
            gkey.push_back({kp, k0p});
        }
    std::vector<int> gorder(groups.size());
    for (size_t i = 0; i < gorder.size(); i++) gorder[i] = (int)i;
    std::stable_sort(gorder.begin(), gorder.end(), [&](int a, int b) { return groups[a].first > groups[b].first; });
    std::vector<int> order;
    for (int gi : gorder) {
        P->kp[P->ngroups] = gkey[gi].first;
        P->k0p[P->ngroups] = gkey[gi].second;
        P->goff[P->ngroups] = (int)order.size();
        P->gcount[P->ngroups] = (int)groups[gi].second.size();
        P->ngroups++;
        order.insert(order.end(), groups[gi].second.begin(), groups[gi].second.end());
    }
    hipStream_t user = (hipStream_t)stream;
    auto fail = [&](int code) {
        destroy(P);
        return code;
    };
#define PCHK(expr)                                                                            \
    do {                                                                                      \
        hipError_t _e = (expr);                                                               \
        if (_e != hipSuccess) return fail(set_err(THO_E_HIP, std::string(#expr) + ": " + hipGetErrorString(_e))); \
    } while (0)
    if (P->count == 0) {
        *plan = P;
        return 0;
    }
    PCHK(hipMalloc((void**)&P->d_inst, inst.size() * sizeof(BatchedInst)));
    PCHK(hipMalloc((void**)&P->d_lv, lv.size() * sizeof(TsqrLevel)));
    PCHK(hipMalloc((void**)&P->d_order, order.size() * sizeof(int)));
    PCHK(hipMalloc((void**)&P->d_counter, tho_plan_s::MAXG * sizeof(int)));
    PCHK(hipStreamCreateWithFlags(&P->cs, hipStreamNonBlocking));
    for (auto& f : P->fork) PCHK(hipStreamCreateWithFlags(&f, hipStreamNonBlocking));
    for (auto& e : P->ev) PCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    // the caller's stream may still be producing the inputs
    hipEvent_t ready;
    PCHK(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
    PCHK(hipEventRecord(ready, user));
    PCHK(hipStreamWaitEvent(P->cs, ready, 0));
    PCHK(hipEventDestroy(ready));
    PCHK(hipMemcpyAsync(P->d_inst, inst.data(), inst.size() * sizeof(BatchedInst), hipMemcpyHostToDevice, P->cs));
    PCHK(hipMemcpyAsync(P->d_lv, lv.data(), lv.size() * sizeof(TsqrLevel), hipMemcpyHostToDevice, P->cs));
    PCHK(hipMemcpyAsync(P->d_order, order.data(), order.size() * sizeof(int), hipMemcpyHostToDevice, P->cs));
    PCHK(hipStreamSynchronize(P->cs));

    // autotune (tile height, persistent workgroups), cached per batch signature
    int dev = 0, cus = 256;
    PCHK(hipGetDevice(&dev));
    PCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    hipDeviceProp_t prop;
    PCHK(hipGetDeviceProperties(&prop, dev));
    std::string arch(prop.gcnArchName);
    for (char& ch : arch)
        if (ch == ' ' || ch == '\n') ch = '_';
    const TuneKey key(arch, cus, P->count, sig_n, sig_k0, sig_k);
    bool cached = false;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_file_load();
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            P->rbo = it->second.first;
            P->grid = it->second.second;
            cached = true;
        }
    }
    if (!cached) {
        hipEvent_t e0, e1;
        PCHK(hipEventCreate(&e0));
        PCHK(hipEventCreate(&e1));
        float best = 1e30f;
        for (int rbo : {4, 2})
            for (int grid : {4 * cus, 3 * cus, 2 * cus, cus}) {
                // one untimed launch (cold caches, first use of the variant),
                // then the best of three
                if (int r = launch_all(P, rbo, grid, P->cs)) return fail(r);
                float t = 1e30f;
                for (int rep = 0; rep < 3; rep++) {
                    PCHK(hipEventRecord(e0, P->cs));
                    if (int r = launch_all(P, rbo, grid, P->cs)) return fail(r);
                    PCHK(hipEventRecord(e1, P->cs));
                    PCHK(hipEventSynchronize(e1));
                    float ms = 0.f;
                    PCHK(hipEventElapsedTime(&ms, e0, e1));
                    t = std::min(t, ms);
                }
                if (t < best) {
                    best = t;
                    P->rbo = rbo;
                    P->grid = grid;
                }
            }
        hipEventDestroy(e0);
        hipEventDestroy(e1);
        P->tuned_ms = best;
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[key] = {P->rbo, P->grid};
        tune_file_append(key, P->rbo, P->grid);
    }
    // capture the launch sequence once
    PCHK(hipStreamBeginCapture(P->cs, hipStreamCaptureModeThreadLocal));
    int lrc = launch_all(P, P->rbo, P->grid, P->cs);
    hipGraph_t g = nullptr;
    hipError_t ec = hipStreamEndCapture(P->cs, &g);
    P->graph = g;
    if (lrc) return fail(lrc);
    PCHK(ec);
    PCHK(hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0));
#undef PCHK
    *plan = P;
    return 0;
}

int tho_batched_run(tho_plan_t plan, void* stream) {
    if (!plan) return set_err(-1, "plan is NULL");
    if (plan->count == 0) return 0;
    PROF("batched", (hipStream_t)stream, hipGraphLaunch(plan->exec, (hipStream_t)stream));
    return 0;
}

int tho_batched_plan_info(tho_plan_t plan, int32_t* tile_rows, int32_t* grid, double* tuned_ms) {
    if (!plan) return set_err(-1, "plan is NULL");
    if (tile_rows) *tile_rows = batched_tile_rows(16, plan->rbo);
    if (grid) *grid = plan->grid;
    if (tuned_ms) *tuned_ms = plan->tuned_ms;
    return 0;
}

int tho_plan_destroy(tho_plan_t plan) {
    destroy(plan);
    return 0;
}

}  // extern "C"
