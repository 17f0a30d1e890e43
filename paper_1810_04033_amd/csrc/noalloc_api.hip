// The residual for callers that cannot allocate device memory: no grid
// handle, no per-call or per-grid scratch.  The first-stage reduction partials
// live in a fixed device array of this file, one copy per device, whose
// address is looked up once per device (with that device current) and then
// passed to the same residual kernels cs_residual runs.
#include <mutex>

#include "cs_internal.h"

using namespace cs;

namespace {

// The residual kernels write at most kMaxResidualBlocks partials (the grid of
// the first stage is clamped to that), each block exactly its own entry, and
// the second stage reads only those: nothing needs clearing between calls.
__device__ __align__(256) Partial scratch[kMaxResidualBlocks];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device dev (the current device).
cs_status scratch_on(int dev, Partial** out)
{
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device %d beyond the %d devices the static scratch serves", dev, kMaxDevices);
        return CS_EUNSUPPORTED;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            set_error("hipGetSymbolAddress of the residual scratch failed on device %d: %s", dev,
                      hipGetErrorString(e));
            return CS_EHIP;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = (Partial*)g_scratch_ptr[dev];
    return CS_OK;
}

}  // namespace

extern "C" {

cs_status cs_residual_noalloc(const cs_grid_desc* desc, const void* u, const void* b, void* r,
                              double* norms, void* stream)
{
    cs_status st = validate_desc_pub(desc);
    if (st != CS_OK) return st;
    if (!norms && !r) { set_error("neither r nor norms given"); return CS_EINVAL; }
    const size_t elem = desc->dtype == CS_F64 ? 8 : 4;
    const size_t bytes = (size_t)span_of_pub(*desc) * elem;
    if ((st = check_device_range_pub(u, bytes, elem, "u")) != CS_OK) return st;
    if ((st = check_device_range_pub(b, bytes, elem, "b")) != CS_OK) return st;
    if (u == b) { set_error("u and b must be separate arrays"); return CS_EINVAL; }
    if (norms && (st = check_device_range_pub(norms, 3 * sizeof(double), sizeof(double), "norms")) != CS_OK)
        return st;
    if (r) {
        if (r == u || r == b) { set_error("r must be a separate array"); return CS_EINVAL; }
        if ((st = check_device_range_pub(r, bytes, elem, "r")) != CS_OK) return st;
    }
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    Partial* partials = nullptr;
    if ((st = scratch_on(dev, &partials)) != CS_OK) return st;
    Geo g;
    g.nx = desc->n[0];
    g.ny = desc->n[1];
    g.nz = desc->dim == 3 ? desc->n[2] : 1;
    g.sy = desc->stride[1];
    g.sz = desc->dim == 3 ? desc->stride[2] : 0;
    g.parity = desc->parity;
    return launch_residual(desc->dtype, desc->dim, desc->stencil, g, u, b, r, desc->h * desc->h,
                           partials, norms, (hipStream_t)stream);
}

}  // extern "C"
