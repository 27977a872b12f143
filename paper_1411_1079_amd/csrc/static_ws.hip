// rh15d_solve_columns_static: the solve with its workspace in a fixed
// device region of the library, for callers that cannot allocate (code
// under graph capture, tight serving loops, harnesses that forbid
// hipMalloc).
//
// The region is a file-scope __device__ array.  In host code its name only
// stands in for the device symbol, so its device address is looked up once
// per device (hipGetSymbolAddress, with that device current) and that
// address is what the kernels receive as their workspace.  Every call on a
// device shares the device's region; the solve's set-up kernel clears the
// slot tables and counters it needs at the start of every call, so no state
// carries over, but calls that overlap on one device race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "rh15d_internal.h"

namespace {

constexpr size_t kStaticWorkspaceBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kStaticWorkspaceBytes];

std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};

// device address of this device's region (looked up on first use)
int scratch_address(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) { rh15d::set_error("hipGetDevice: %s", hipGetErrorString(e)); return RH15D_EDEVICE; }
    if (dev < 0 || dev >= kMaxDevices) { rh15d::set_error("device %d beyond %d", dev, kMaxDevices); return RH15D_EDEVICE; }
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            rh15d::set_error("hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
            return RH15D_EDEVICE;
        }
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return RH15D_OK;
}

}  // namespace

extern "C" {

size_t rh15d_static_workspace_bytes(void) { return kStaticWorkspaceBytes; }

int rh15d_solve_columns_static(const rh15d_atom *atom, const rh15d_columns *cols, const rh15d_options *opt,
                               const rh15d_outputs *out, void *hip_stream) {
    void *ws = nullptr;
    int rc = scratch_address(&ws);
    if (rc != RH15D_OK) return rc;
    return rh15d::solve_columns_impl(atom, cols, opt, out, ws, kStaticWorkspaceBytes, hip_stream, true);
}

}  // extern "C"
