// Kernels and launchers of the chunked tall-skinny Householder QR and of the
// formation of Q (device code in tsqr_dev.h).
#include "tsqr_dev.h"

namespace tho {

template <int KP, int K0P, int PANEL>
__global__ __launch_bounds__(NW * 64, 2) void k_tsqr_leaf(TsqrLevel L) {
    leaf_chunk<KP, K0P, PANEL, 0>(L, blockIdx.x);
}

template <int KP, int K0P, int PANEL>
__global__ __launch_bounds__(NW * 64, 2) void k_tsqr_form(TsqrLevel L) {
    form_chunk<KP, K0P, PANEL, 0>(L, blockIdx.x);
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

template <int KP, int K0P, int PANEL>
static hipError_t form_t(const TsqrLevel& L, hipStream_t st) {
    const size_t shm = FormLds<KP>::total * sizeof(double);
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void*)k_tsqr_form<KP, K0P, PANEL>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL((k_tsqr_form<KP, K0P, PANEL>), dim3(L.nchunk), dim3(NW * 64), shm, st, L);
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

hipError_t launch_tsqr_leaf(int kp, int k0p, int panel, const TsqrLevel& L, hipStream_t st) {
    if (panel == PANEL_F32X2) TSQR_DISPATCH_LOWP(leaf_t, PANEL_F32X2)
    if (panel == PANEL_BF16) TSQR_DISPATCH_LOWP(leaf_t, PANEL_BF16)
    TSQR_DISPATCH(leaf_t)
}

hipError_t launch_tsqr_form(int kp, int k0p, int panel, const TsqrLevel& L, hipStream_t st) {
    if (panel == PANEL_F32X2) TSQR_DISPATCH_LOWP(form_t, PANEL_F32X2)
    if (panel == PANEL_BF16) TSQR_DISPATCH_LOWP(form_t, PANEL_BF16)
    TSQR_DISPATCH(form_t)
}

}  // namespace tho
