// lb_noalloc.hip -- the trace misfit with no workspace argument, for callers
// that cannot allocate device memory: code under HIP graph capture, tight
// serving loops and harnesses that forbid hipMalloc.  It is lb_trace_misfit
// with the FP64 block partials in a file-scope device array instead of a
// caller workspace; the kernels are the same, so the results are the same
// bits.  Nothing here allocates: the array is part of the code object, one
// copy per GPU, held until the process ends.
#include "lbwave.h"
#include "lb_host.h"
#include "lb_internal.h"

#include <mutex>

namespace {

// One FP64 partial per block of the misfit's grid-stride loop (at most
// kMisfitMaxBlocks blocks): 16 KiB per GPU.  Every call writes each slot it
// reads before reading it, so nothing needs clearing between calls.
__device__ __align__(256) double scratch[lbw::kMisfitMaxBlocks];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double *g_scratch[kMaxDevices] = {};

// The device address of `scratch` on the GPU that runs `stream` (the
// current device for the null stream), taken once per device with that
// device current.  In host code the name `scratch` is only a stand-in; the
// kernels get this address.
int scratch_for_stream(hipStream_t stream, double **out) {
    int dev = -1;
    if (stream != nullptr) {
        if (hipStreamGetDevice(stream, &dev) != hipSuccess) return LB_E_HIP;
    } else if (hipGetDevice(&dev) != hipSuccess) {
        return LB_E_HIP;
    }
    if (dev < 0 || dev >= kMaxDevices) return LB_E_HIP;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        int cur = -1;
        if (hipGetDevice(&cur) != hipSuccess) return LB_E_HIP;
        if (cur != dev && hipSetDevice(dev) != hipSuccess) return LB_E_HIP;
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev && hipSetDevice(cur) != hipSuccess) return LB_E_HIP;
        if (e != hipSuccess || p == nullptr) return LB_E_HIP;
        g_scratch[dev] = static_cast<double *>(p);
    }
    *out = g_scratch[dev];
    return LB_OK;
}

}  // namespace

extern "C" int lb_trace_misfit_static(const void *d_traces, const void *d_obs, void *d_res, int32_t nrec, int64_t cap,
                                      int64_t ncols, lb_dtype t, double *d_phi, void *stream) {
    int rc = lbw::check_trace_misfit(d_traces, d_obs, d_res, nrec, cap, ncols, t, d_phi);
    if (rc) return rc;
    double *partial = nullptr;
    if ((rc = scratch_for_stream(static_cast<hipStream_t>(stream), &partial))) return rc;
    return lbw::launch_misfit(t == LB_F64 ? lbw::ST_F64 : lbw::ST_F32, d_traces, d_obs, d_res, nrec, cap, ncols, d_phi,
                              partial, static_cast<hipStream_t>(stream)) == hipSuccess ? LB_OK : LB_E_HIP;
}
