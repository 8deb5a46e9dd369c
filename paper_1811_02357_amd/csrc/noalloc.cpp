// noalloc.cpp -- irtps_solve_static: the whole IRT-PS solve in a device scratch
// area that the library owns, for callers that cannot allocate device memory.
//
// The scratch is a file-scope device array (one copy on every GPU the library
// runs on, held until the process ends).  Its device address is looked up once
// per device, on the entry point's first call there with that device current;
// the array's name is a host-side stand-in and is never handed to a kernel or a
// copy.  Every call on a GPU uses the same array: calls that overlap on one GPU
// race.  The solve needs no initialised workspace (every buffer it reads in a
// call is written earlier in that call), so nothing is cleared between calls.
#include <hip/hip_runtime.h>

#include <mutex>

#include "host.hpp"
#include "irtps.h"

using namespace irtps;
using namespace irtps::host;

namespace {

constexpr size_t kScratchBytes = IRTPS_STATIC_SCRATCH_BYTES;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};  // per device: the array's device address

// The device address of this device's scratch (looked up on first use).
int scratch_of_current_device(void** out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return IRTPS_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p || (reinterpret_cast<uintptr_t>(p) % kAlign)) return IRTPS_ERR_DEVICE;
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return IRTPS_OK;
}

}  // namespace

extern "C" int irtps_solve_static(const irtps_problem* problem, const irtps_params* params,
                                  const irtps_outputs* outputs, void* stream) {
    size_t need = 0;
    STATUS_TRY(irtps_workspace_bytes(problem, params, &need));
    if (need > kScratchBytes) return IRTPS_ERR_WORKSPACE;
    void* ws = nullptr;
    STATUS_TRY(scratch_of_current_device(&ws));
    // the tracer's optional timing events are created per launch: off here
    const bool prof = g_prof.on;
    g_prof.on = false;
    const int rc = irtps_solve(problem, params, outputs, ws, kScratchBytes, stream);
    g_prof.on = prof;
    return rc;
}
