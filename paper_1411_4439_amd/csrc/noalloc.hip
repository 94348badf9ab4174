// hisq_cg_solve_noalloc: the CG solve of hisq_cg_solve for callers that cannot
// allocate device memory or pass a workspace.  Every device region the solve
// needs beyond the caller's links, b and x (CG scalars, reduction partials and
// counters, the working fields) lives in one file-scope device array.
//
// The array is one object per GPU: the runtime places a copy on every device
// that loads this code object, at its own address.  In host code the array's
// name is only a stand-in for the symbol, never a device address, so the
// address of each device's copy is looked up once per device with
// hipGetSymbolAddress (with that device current) and only that address is
// handed to kernels.
#include <cstdio>
#include <mutex>

#include "hisq_internal.h"

namespace hisq {

constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
constexpr int kNoAllocMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

std::mutex g_scratch_mu;
void* g_scratch_ptr[kNoAllocMaxDevices] = {};

// Device address of the current device's scratch array, looked up on the
// first call on that device.
hipError_t device_scratch(void** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kNoAllocMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

// Host copies of the CG state: ordinary host memory of the calling thread
// (the allocating entry points use a pinned buffer).
thread_local CgState t_host_states[HISQ_MAX_PROBLEMS];

}  // namespace

}  // namespace hisq

using namespace hisq;

extern "C" {

int hisq_cg_solve_noalloc(const hisq_geom* g, double mass, int nrhs, const hisq_params* p,
                          const void* links64, const void* links32, const double* b_e,
                          double* x_e, hisq_info* info, void* stream)
{
    (void)hipGetLastError();  // drop a stale error left by an earlier failed call
    static_assert(kNoAllocScratchBytes == HISQ_NOALLOC_SCRATCH_BYTES, "documented limit");
    if (!p)  // the solve's own checks report it
        return cg_solve_on(g, mass, nrhs, p, links64, links32, b_e, x_e, nullptr, 0, info, stream,
                           t_host_states);
    // 0 for an invalid geometry, bundle or mode: the solve's checks report those
    const size_t need = hisq_workspace_bytes(g, nrhs, p->mode);
    if (need > kNoAllocScratchBytes)
        return report_error(HISQ_EWORKSPACE,
                            "hisq_cg_solve_noalloc: this solve needs %zu bytes of scratch, the "
                            "static scratch array holds %zu (use hisq_cg_solve with a workspace)",
                            need, kNoAllocScratchBytes);
    void* ws = nullptr;
    const hipError_t e = device_scratch(&ws);
    if (e != hipSuccess)
        return report_error(HISQ_EHIP, "hisq_cg_solve_noalloc: scratch address lookup failed: %s",
                            hipGetErrorString(e));
    // no hipGraph (instantiating one may allocate) and no profiling events
    hisq_params q = *p;
    q.use_graph = 0;
    q.profile = 0;
    return cg_solve_on(g, mass, nrhs, &q, links64, links32, b_e, x_e, ws, kNoAllocScratchBytes,
                       info, stream, t_host_states);
}

}  // extern "C"
