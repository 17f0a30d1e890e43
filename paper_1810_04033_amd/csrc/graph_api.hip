// Captured sweep sequences: a fixed number of sweeps of one grid or one batch
// recorded once into a HIP graph and replayed with a single launch call,
// which removes the per-kernel launch cost that dominates small grids, the
// one-launch-per-colour passes and the hyperplane wavefronts.  Only kernel
// nodes are recorded (the sweep paths issue no memset or copy calls).
#include "cs_internal.h"

#include <new>

struct cs_graph_s {
    hipGraph_t graph;
    hipGraphExec_t exec;
    int device;
};

namespace {

using cs::hip_fail;
using cs::set_error;

template <typename F>
cs_status capture(F&& record, cs_graph* out)
{
    if (!out) { set_error("NULL output handle"); return CS_EINVAL; }
    *out = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    hipStream_t cs_stream = nullptr;
    if ((e = hipStreamCreateWithFlags(&cs_stream, hipStreamNonBlocking)) != hipSuccess)
        return hip_fail(e, "hipStreamCreateWithFlags");
    if ((e = hipStreamBeginCapture(cs_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
        (void)hipStreamDestroy(cs_stream);
        return hip_fail(e, "hipStreamBeginCapture");
    }
    const cs_status rec = record(cs_stream);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(cs_stream, &graph);
    (void)hipStreamDestroy(cs_stream);
    if (rec != CS_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rec;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t exec = nullptr;
    if ((e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0)) != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return hip_fail(e, "hipGraphInstantiate");
    }
    cs_graph_s* h = new (std::nothrow) cs_graph_s{graph, exec, dev};
    if (!h) {
        (void)hipGraphExecDestroy(exec);
        (void)hipGraphDestroy(graph);
        set_error("out of host memory");
        return CS_ENOMEM;
    }
    *out = h;
    return CS_OK;
}

}  // namespace

extern "C" {

cs_status cs_graph_gs(cs_grid g, int32_t nsweeps, void* u_tmp, int32_t lexicographic, cs_graph* out)
{
    if (!g) { set_error("grid is NULL"); return CS_EINVAL; }
    if (nsweeps < 1) { set_error("nsweeps must be >= 1"); return CS_EINVAL; }
    if (lexicographic != 0 && lexicographic != 1) {
        set_error("lexicographic must be 0 or 1");
        return CS_EINVAL;
    }
    if (lexicographic && u_tmp) { set_error("the lexicographic sweep takes no work array"); return CS_EINVAL; }
    return capture([&](hipStream_t s) {
        return lexicographic ? cs_gs_sweeps_lex(g, nsweeps, s) : cs_gs_sweeps(g, nsweeps, u_tmp, s);
    }, out);
}

cs_status cs_graph_batch_gs(cs_batch bt, int32_t nsweeps, cs_graph* out)
{
    if (!bt) { set_error("batch is NULL"); return CS_EINVAL; }
    if (nsweeps < 1) { set_error("nsweeps must be >= 1"); return CS_EINVAL; }
    return capture([&](hipStream_t s) { return cs_batch_gs_sweeps(bt, nsweeps, s); }, out);
}

cs_status cs_graph_launch(cs_graph gr, void* stream)
{
    if (!gr) { set_error("graph is NULL"); return CS_EINVAL; }
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev != gr->device) {
        set_error("graph was captured on device %d, current device is %d", gr->device, dev);
        return CS_EINVAL;
    }
    if ((e = hipGraphLaunch(gr->exec, (hipStream_t)stream)) != hipSuccess)
        return hip_fail(e, "hipGraphLaunch");
    return CS_OK;
}

cs_status cs_graph_destroy(cs_graph gr)
{
    if (!gr) return CS_OK;
    hipError_t e1 = hipGraphExecDestroy(gr->exec);
    hipError_t e2 = hipGraphDestroy(gr->graph);
    delete gr;
    if (e1 != hipSuccess) return hip_fail(e1, "hipGraphExecDestroy");
    if (e2 != hipSuccess) return hip_fail(e2, "hipGraphDestroy");
    return CS_OK;
}

}  // extern "C"
