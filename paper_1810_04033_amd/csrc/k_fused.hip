// Fused single-pass Gauss-Seidel sweeps (placeholder until the kernels land).
#include "cs_device.h"
#include "cs_internal.h"

namespace cs {

bool fused_supported(int, int, int, const Geo&) { return false; }

cs_status launch_fused_sweep(int, int, int, const Geo&, const void*, void*, const void*, double,
                             hipStream_t)
{
    set_error("fused sweep not available for this grid");
    return CS_EUNSUPPORTED;
}

}  // namespace cs
