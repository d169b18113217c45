// fld_step without any allocation: for callers that cannot allocate device or
// pinned memory (code under HIP graph capture, tight serving loops, harnesses
// that forbid it).  The plan's tables and multigrid fields live in a fixed
// device array of this library, `scratch`, instead of a caller workspace.
//
// The array is a file-scope __device__ variable: each GPU the library runs on
// holds its own copy until the process ends, at its own address.  Host code never
// names it directly (in host code the name is a host-side stand-in, not a device
// address): at the first call on a device, with that device current, its address
// is taken with hipGetSymbolAddress and kept per device; the step uses that
// address.  Every call on a device shares the one array, so calls that overlap on
// one GPU race; each call rebinds its plan's tables into the array, and no kernel
// of the step expects any part of it to start at zero.
#include "fld_internal.hpp"

#include <mutex>

namespace fld {
namespace {

constexpr size_t kScratchBytes = (size_t)FLD_NOALLOC_MAX_BYTES;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of this device's copy of `scratch` (taken once per device).
int scratch_address(int dev, void** out) {
    if (dev < 0 || dev >= kMaxDevices) return FLD_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            set_error("hipGetSymbolAddress(scratch)", e != hipSuccess ? e : hipErrorInvalidSymbol);
            return FLD_ERR_HIP;
        }
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return FLD_OK;
}

}  // namespace
}  // namespace fld

extern "C" int32_t fld_step_noalloc(fld_plan_t plan, const double* const* E_in, const double* const* kappa_rho,
                                    double* const* E_out, const double* dt, void* stream, fld_stats* stats) {
    fld::Plan* p = fld::plan_of(plan);
    if (!p || !E_in || !kappa_rho || !E_out || !dt) return FLD_ERR_INVALID_ARG;
    try {
        int prev = -1;
        if (hipGetDevice(&prev) != hipSuccess) return FLD_ERR_HIP;
        if (prev != p->device && hipSetDevice(p->device) != hipSuccess) return FLD_ERR_HIP;
        void* ptr = nullptr;
        int rc = fld::scratch_address(p->device, &ptr);
        hipStream_t s = static_cast<hipStream_t>(stream);
        if (rc == FLD_OK && hipStreamSynchronize(s) != hipSuccess) rc = FLD_ERR_HIP;
        if (rc == FLD_OK) rc = fld::plan_step_noalloc(*p, ptr, fld::kScratchBytes, E_in, kappa_rho, E_out, dt, s, stats);
        if (prev != p->device) (void)hipSetDevice(prev);
        return rc;
    } catch (...) {
        return FLD_ERR_INVALID_ARG;
    }
}
