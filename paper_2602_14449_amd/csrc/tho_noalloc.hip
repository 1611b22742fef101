// tho_two_stage_noalloc: the two-stage orthogonalization (Algorithm 1, second
// choice of P) for callers that cannot allocate device memory.  The work
// buffer of tho_two_stage is replaced by one file-scope device array per GPU,
// `scratch`, of THO_NOALLOC_SCRATCH_BYTES bytes; the launch sequence and the
// kernels are those of tho_two_stage.
//
// In host code `scratch` names a host-side stand-in, not device memory: its
// device address is taken once per device with hipGetSymbolAddress (with
// that device current) and only that address is ever handed to kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "tho_host.h"

namespace {

static __device__ __align__(256) unsigned char scratch[THO_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of this device's `scratch` (set up on the first call on
// the device).  Also creates, for this host thread and device, the side
// stream and events the launch sequence forks onto, so that later calls
// create nothing.
int scratch_for_current_device(void** out) {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return tho::set_err(THO_E_UNSUPPORTED, "device ordinal out of range");
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!g_ptr[dev]) {
            void* p = nullptr;
            HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
            if (!p) return tho::set_err(THO_E_HIP, "hipGetSymbolAddress returned a null scratch address");
            g_ptr[dev] = p;
        }
        *out = g_ptr[dev];
    }
    if (!tho::fork_for_thread().ok) return tho::set_err(THO_E_HIP, "could not create the side stream");
    return 0;
}

}  // namespace

int tho::noalloc_scratch(const void** out) {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_mu);
    if (dev < 0 || dev >= kMaxDevices || !g_ptr[dev])
        return tho::set_err(THO_E_UNSUPPORTED, "tho_two_stage_noalloc has not run on this device");
    *out = g_ptr[dev];
    return 0;
}

extern "C" int tho_two_stage_noalloc(int32_t dtype, int64_t n, int64_t k0, int64_t k, const void* V, int64_t ldv,
                                     const void* A, int64_t lda, void* Q, int64_t ldq, void* R, int64_t ldr,
                                     void* S, int64_t lds, const tho_opts_t* opts, void* stream) {
    if (opts && (opts->panel < THO_PANEL_F64 || opts->panel > THO_PANEL_BF16))
        return tho::set_err(-15, "unknown panel precision");
    size_t need = 0;
    int rc = tho_two_stage_workspace(dtype, n, k0, k, opts, &need);
    if (rc) return rc;
    if (need > (size_t)THO_NOALLOC_SCRATCH_BYTES)
        return tho::set_err(THO_E_WORKSPACE, "tho_two_stage_noalloc: these sizes need " + std::to_string(need) +
                                                 " bytes of scratch, above the fixed maximum of " +
                                                 std::to_string((size_t)THO_NOALLOC_SCRATCH_BYTES) +
                                                 " (use tho_two_stage with a caller workspace)");
    if (k == 0) return tho_two_stage(dtype, n, k0, k, V, ldv, A, lda, Q, ldq, R, ldr, S, lds, opts, nullptr, 0,
                                     stream);
    void* ws = nullptr;
    if ((rc = scratch_for_current_device(&ws))) return rc;
    return tho_two_stage(dtype, n, k0, k, V, ldv, A, lda, Q, ldq, R, ldr, S, lds, opts, ws,
                         (size_t)THO_NOALLOC_SCRATCH_BYTES, stream);
}
