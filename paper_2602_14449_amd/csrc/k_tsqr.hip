// Kernels and launchers of the chunked tall-skinny Householder QR and of the
// formation of Q (device code in tsqr_dev.h).
#include "tsqr_dev.h"

namespace tho {

template <int KP, int K0P, int PANEL>
__global__ __launch_bounds__(NW * 64, 2) void k_tsqr_leaf(TsqrLevel L) {
    leaf_chunk<KP, K0P, PANEL, 0>(L, blockIdx.x);
}


// Levels above 0 (no V term): eight wavefronts per chunk, so that a tile
// stacks four R factors of the level below (fan-in 4, half the levels).
constexpr int NW_UP = 8;

template <int KP>
__global__ __launch_bounds__(NW_UP * 64, 1) void k_tsqr_leaf_up(TsqrLevel L) {
    leaf_chunk<KP, 0, 0, 0, NW_UP>(L, blockIdx.x);
}

template <int KP>
__global__ __launch_bounds__(NW_UP * 64, 1) void k_tsqr_form_up(TsqrLevel L) {
    form_chunk<KP, 0, 0, 0, NW_UP>(L, blockIdx.x);
}

template <int KP>
__global__ __launch_bounds__(NW * 64, 2) void k_tsqr_kchain(TsqrLevel L) {
    kchain_chunk<KP>(L, blockIdx.x);
}

// one workgroup per tile slot (chunk-major, so that consecutive workgroups
// stream consecutive rows)
template <int KP, int K0P, int PANEL>
__global__ __launch_bounds__(NW * 64, 2) void k_tsqr_rows(TsqrLevel L) {
    rows_tile<KP, K0P, PANEL>(L, blockIdx.x / L.maxtiles, blockIdx.x % L.maxtiles);
}

// ---------------------------------------------------------------- launchers

template <int KP, int K0P, int PANEL>
static hipError_t leaf_t(const TsqrLevel& L, hipStream_t st) {
    const size_t shm = LeafLds<KP>::total * sizeof(double);
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void*)k_tsqr_leaf<KP, K0P, PANEL>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL((k_tsqr_leaf<KP, K0P, PANEL>), dim3(L.nchunk), dim3(NW * 64), shm, st, L);
    return hipGetLastError();
}

template <int KP>
static hipError_t leaf_up_t(const TsqrLevel& L, hipStream_t st) {
    const size_t shm = LeafLds<KP, 0, NW_UP>::total * sizeof(double);
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void*)k_tsqr_leaf_up<KP>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)shm);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL((k_tsqr_leaf_up<KP>), dim3(L.nchunk), dim3(NW_UP * 64), shm, st, L);
    return hipGetLastError();
}

template <int KP>
static hipError_t form_up_t(const TsqrLevel& L, hipStream_t st) {
    const size_t shm = FormLds<KP>::total * sizeof(double);
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void*)k_tsqr_form_up<KP>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)shm);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL((k_tsqr_form_up<KP>), dim3(L.nchunk), dim3(NW_UP * 64), shm, st, L);
    return hipGetLastError();
}

template <int KP>
static hipError_t kchain_t(const TsqrLevel& L, hipStream_t st) {
    const size_t shm = KchainLds<KP>::total * sizeof(double);
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void*)k_tsqr_kchain<KP>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL((k_tsqr_kchain<KP>), dim3(L.nchunk), dim3(NW * 64), shm, st, L);
    return hipGetLastError();
}

template <int KP, int K0P, int PANEL>
static hipError_t rows_t(const TsqrLevel& L, hipStream_t st) {
    const int64_t nb = (int64_t)L.nchunk * L.maxtiles;
    if (nb <= 0 || nb > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_tsqr_rows<KP, K0P, PANEL>), dim3((unsigned)nb), dim3(NW * 64), 0, st, L);
    return hipGetLastError();
}

#define TSQR_DISPATCH(FN)                                  \
    switch (kp * 1000 + k0p) {                             \
        case 16000: return FN<16, 0, 0>(L, st);            \
        case 16016: return FN<16, 16, 0>(L, st);           \
        case 16032: return FN<16, 32, 0>(L, st);           \
        case 16064: return FN<16, 64, 0>(L, st);           \
        case 16128: return FN<16, 128, 0>(L, st);          \
        case 32000: return FN<32, 0, 0>(L, st);            \
        case 32016: return FN<32, 16, 0>(L, st);           \
        case 32032: return FN<32, 32, 0>(L, st);           \
        case 32064: return FN<32, 64, 0>(L, st);           \
        case 32128: return FN<32, 128, 0>(L, st);          \
        case 64000: return FN<64, 0, 0>(L, st);            \
        case 64016: return FN<64, 16, 0>(L, st);           \
        case 64032: return FN<64, 32, 0>(L, st);           \
        case 64064: return FN<64, 64, 0>(L, st);           \
        case 64128: return FN<64, 128, 0>(L, st);          \
        default: return hipErrorInvalidValue;              \
    }

// reduced-precision panels exist only with a V term (k0p > 0)
#define TSQR_DISPATCH_LOWP(FN, P)                          \
    switch (kp * 1000 + k0p) {                             \
        case 16016: return FN<16, 16, P>(L, st);           \
        case 16032: return FN<16, 32, P>(L, st);           \
        case 16064: return FN<16, 64, P>(L, st);           \
        case 16128: return FN<16, 128, P>(L, st);          \
        case 32016: return FN<32, 16, P>(L, st);           \
        case 32032: return FN<32, 32, P>(L, st);           \
        case 32064: return FN<32, 64, P>(L, st);           \
        case 32128: return FN<32, 128, P>(L, st);          \
        case 64016: return FN<64, 16, P>(L, st);           \
        case 64032: return FN<64, 32, P>(L, st);           \
        case 64064: return FN<64, 64, P>(L, st);           \
        case 64128: return FN<64, 128, P>(L, st);          \
        default: return hipErrorInvalidValue;              \
    }

#ifdef THO_PHASE_TIMING
extern "C" int tho_debug_phase_read(long long* out, int n) {
    return (int)hipMemcpyFromSymbol(out, HIP_SYMBOL(g_phase_ts), sizeof(long long) * n, 0, hipMemcpyDeviceToHost);
}
#endif

int tsqr_tile_rows(int kp) {
    return kp >= 64 ? Geo<64>::TB : Geo<16>::TB;
}

int tsqr_tile_rows_up(int kp) {
    return kp >= 64 ? Geo<64, 0, NW_UP>::TB : Geo<16, 0, NW_UP>::TB;
}

hipError_t launch_tsqr_leaf(int kp, int k0p, int panel, const TsqrLevel& L, hipStream_t st) {
    if (panel == PANEL_F32X2) TSQR_DISPATCH_LOWP(leaf_t, PANEL_F32X2)
    if (panel == PANEL_BF16) TSQR_DISPATCH_LOWP(leaf_t, PANEL_BF16)
    TSQR_DISPATCH(leaf_t)
}

hipError_t launch_tsqr_leaf_up(int kp, const TsqrLevel& L, hipStream_t st) {
    switch (kp) {
        case 16: return leaf_up_t<16>(L, st);
        case 32: return leaf_up_t<32>(L, st);
        case 64: return leaf_up_t<64>(L, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_tsqr_form_up(int kp, const TsqrLevel& L, hipStream_t st) {
    switch (kp) {
        case 16: return form_up_t<16>(L, st);
        case 32: return form_up_t<32>(L, st);
        case 64: return form_up_t<64>(L, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_tsqr_kchain(int kp, const TsqrLevel& L, hipStream_t st) {
    if (L.Cfin == nullptr) return hipErrorInvalidValue;
    switch (kp) {
        case 16: return kchain_t<16>(L, st);
        case 32: return kchain_t<32>(L, st);
        case 64: return kchain_t<64>(L, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_tsqr_rows(int kp, int k0p, int panel, const TsqrLevel& L, hipStream_t st) {
    if (L.Cfin == nullptr) return hipErrorInvalidValue;
    if (panel == PANEL_F32X2) TSQR_DISPATCH_LOWP(rows_t, PANEL_F32X2)
    if (panel == PANEL_BF16) TSQR_DISPATCH_LOWP(rows_t, PANEL_BF16)
    TSQR_DISPATCH(rows_t)
}

}  // namespace tho
