// Captured sweep sequences: a fixed number of sweeps of one grid or one batch,
// or any sequence of library calls the caller enqueues between cs_graph_begin
// and cs_graph_end, recorded once into a HIP graph and replayed with a single
// launch call,
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

// Start a thread-local capture on a fresh non-blocking stream of the library.
cs_status begin_capture(hipStream_t* out)
{
    *out = nullptr;
    hipStream_t cs_stream = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "hipStreamCreateWithFlags");
    if ((e = hipStreamBeginCapture(cs_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
        (void)hipStreamDestroy(cs_stream);
        return hip_fail(e, "hipStreamBeginCapture");
    }
    *out = cs_stream;
    return CS_OK;
}

// End the capture on cs_stream, release the stream, and (if rec is CS_OK)
// instantiate the graph into *out.
cs_status end_capture(hipStream_t cs_stream, cs_status rec, cs_graph* out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    hipGraph_t graph = nullptr;
    const hipError_t ee = hipStreamEndCapture(cs_stream, &graph);
    (void)hipStreamDestroy(cs_stream);
    if (rec != CS_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rec;
    }
    if (ee != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return hip_fail(ee, "hipStreamEndCapture");
    }
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return hip_fail(e, "hipGetDevice");
    }
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

template <typename F>
cs_status capture(F&& record, cs_graph* out)
{
    if (!out) { set_error("NULL output handle"); return CS_EINVAL; }
    *out = nullptr;
    hipStream_t cs_stream = nullptr;
    cs_status st = begin_capture(&cs_stream);
    if (st != CS_OK) return st;
    return end_capture(cs_stream, record(cs_stream), out);
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

cs_status cs_graph_begin(void** capture_stream)
{
    if (!capture_stream) { set_error("NULL output stream"); return CS_EINVAL; }
    hipStream_t st = nullptr;
    cs_status rc = begin_capture(&st);
    *capture_stream = st;
    return rc;
}

cs_status cs_graph_end(void* capture_stream, cs_graph* out)
{
    if (!capture_stream || !out) { set_error("NULL argument"); return CS_EINVAL; }
    *out = nullptr;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing((hipStream_t)capture_stream, &cap);
    if (e != hipSuccess) return hip_fail(e, "hipStreamIsCapturing");
    if (cap == hipStreamCaptureStatusNone) {
        set_error("stream is not capturing");
        return CS_EINVAL;
    }
    return end_capture((hipStream_t)capture_stream, CS_OK, out);
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
