// noalloc.hip -- intsort_sort_keys_noalloc: the key sort for callers that
// cannot allocate (code under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc).  Its workspace is the library's own
// device array `scratch` of NOALLOC_SCRATCH_BYTES, one copy per device,
// held until the process ends.  Every call on a device shares that device's
// copy: calls that overlap on one device race (the sort's first kernels
// clear the counters, histograms and look-back words it reads, so a call
// never depends on what an earlier call left).
#include <hip/hip_runtime.h>

#include <mutex>

#include "intsort.h"
#include "internal.hpp"

namespace {

constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)INTSORT_NOALLOC_SCRATCH_MB << 20;

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_lock;
void *g_scratch[MAX_DEVICES];   // device address of `scratch` on each device, once known

}  // namespace

namespace intsort {

// Takes the device address of `scratch` on `device` (which must be the
// current device).  In host code `scratch` names a host-side stand-in; only
// this address may reach a kernel or a copy.
hipError_t noalloc_setup(int device)
{
    if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(g_lock);
    if (g_scratch[device]) return hipSuccess;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (p == nullptr || (reinterpret_cast<uintptr_t>(p) & 255u) != 0) return hipErrorInvalidValue;
    g_scratch[device] = p;
    return hipSuccess;
}

}  // namespace intsort

extern "C" intsort_status intsort_sort_keys_noalloc(intsort_ctx *ctx, intsort_key_type kt, const void *keys_in,
                                                   void *keys_out, uint64_t n, const intsort_options *opts,
                                                   void *stream)
{
    try {
        if (!ctx) return INTSORT_ERR_INVALID_ARGUMENT;
        size_t need = 0;
        intsort_status st = intsort_workspace_size(ctx, kt, 0, n, 0, opts, &need);
        if (st != INTSORT_OK) return st;
        if (need > NOALLOC_SCRATCH_BYTES) return INTSORT_ERR_WORKSPACE_TOO_SMALL;
        const int device = intsort::ctx_device(ctx);
        void *ws = nullptr;
        if (device >= 0 && device < MAX_DEVICES) {
            std::lock_guard<std::mutex> g(g_lock);
            ws = g_scratch[device];
        }
        // a planning context, or a device whose address was not taken at
        // intsort_create: the sort call reports it (unsupported / invalid)
        if (!ws && device >= 0) return INTSORT_ERR_INTERNAL;
        return intsort_sort_keys(ctx, kt, keys_in, keys_out, n, opts, ws, ws ? NOALLOC_SCRATCH_BYTES : 0, stream);
    } catch (...) {
        return INTSORT_ERR_INTERNAL;
    }
}
