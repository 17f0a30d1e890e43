// C ABI of the colsten library: argument validation, dispatch and the sweep
// drivers.  No function here synchronises the host except the create calls.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <cmath>
#include <cstdint>
#include <new>

#include "cs_internal.h"

namespace cs {

namespace {
thread_local char g_err[512] = "";
}

void set_error(const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}

cs_status hip_fail(hipError_t e, const char* what)
{
    set_error("%s: %s", what, hipGetErrorString(e));
    return CS_EHIP;
}

cs_status check_launch(const char* what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, what);
    return CS_OK;
}

namespace {

int64_t span_of(const cs_grid_desc& d)
{
    if (d.dim == 2) return (d.n[1] + 1) * d.stride[1] + d.n[0] + 2;
    return (d.n[2] + 1) * d.stride[2] + (d.n[1] + 1) * d.stride[1] + d.n[0] + 2;
}

cs_status validate_desc(const cs_grid_desc* d)
{
    if (!d) { set_error("desc is NULL"); return CS_EINVAL; }
    if (d->dim != 2 && d->dim != 3) { set_error("dim must be 2 or 3 (got %d)", d->dim); return CS_EINVAL; }
    if (d->stencil != CS_FD && d->stencil != CS_Q1) { set_error("unknown stencil %d", d->stencil); return CS_EINVAL; }
    if (d->dtype != CS_F64 && d->dtype != CS_F32) { set_error("unknown dtype %d", d->dtype); return CS_EINVAL; }
    if (d->parity != 0 && d->parity != 1) { set_error("parity must be 0 or 1"); return CS_EINVAL; }
    const int64_t lim = (int64_t)1 << 24;
    for (int a = 0; a < d->dim; ++a)
        if (d->n[a] < 1 || d->n[a] > lim) { set_error("n[%d] = %lld out of range [1, 2^24]", a, (long long)d->n[a]); return CS_EINVAL; }
    if (d->dim == 2 && d->n[2] != 1) { set_error("n[2] must be 1 for a 2D grid"); return CS_EINVAL; }
    if (d->stride[0] != 1) { set_error("stride[0] must be 1 (x contiguous)"); return CS_EINVAL; }
    if (d->stride[1] < d->n[0] + 2) { set_error("stride[1] must be >= n[0] + 2"); return CS_EINVAL; }
    if (d->dim == 3 && d->stride[2] < d->stride[1] * (d->n[1] + 2)) {
        set_error("stride[2] must be >= stride[1] * (n[1] + 2)");
        return CS_EINVAL;
    }
    if (!(d->h > 0.0) || !std::isfinite(d->h)) { set_error("h must be finite and > 0"); return CS_EINVAL; }
    const double total = (double)span_of(*d);
    if (total > 9.0e18 / 8) { set_error("grid extent overflows"); return CS_EINVAL; }
    return CS_OK;
}

// The pointer must be device memory on the current device, aligned to the
// element size, and the allocation must cover `bytes` from it.
cs_status check_device_range(const void* p, size_t bytes, size_t align, const char* name,
                             size_t* room_before = nullptr, size_t* room_after = nullptr)
{
    if (!p) { set_error("%s is NULL", name); return CS_EINVAL; }
    if ((uintptr_t)p % align) { set_error("%s is not %zu-byte aligned", name, align); return CS_EINVAL; }
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    hipPointerAttribute_t attr;
    e = hipPointerGetAttributes(&attr, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        set_error("%s is not a HIP allocation", name);
        return CS_EINVAL;
    }
    if (attr.type != hipMemoryTypeDevice) { set_error("%s is not device memory", name); return CS_EINVAL; }
    if (attr.device != dev) { set_error("%s lives on device %d, current device is %d", name, attr.device, dev); return CS_EINVAL; }
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    e = hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        set_error("%s: cannot query its allocation range", name);
        return CS_EINVAL;
    }
    const uintptr_t lo = (uintptr_t)base, hi = lo + size, a = (uintptr_t)p;
    if (a < lo || a + bytes > hi) {
        set_error("%s: the halo'd grid (%zu bytes) runs past its allocation", name, bytes);
        return CS_EINVAL;
    }
    if (room_before) *room_before = a - lo;
    if (room_after) *room_after = hi - (a + bytes);
    return CS_OK;
}

cs_status check_grid(cs_grid g)
{
    if (!g) { set_error("grid is NULL"); return CS_EINVAL; }
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev != g->device) { set_error("grid belongs to device %d, current device is %d", g->device, dev); return CS_EINVAL; }
    return CS_OK;
}

double h2_of(const cs_grid_s* g)
{
    const double h2 = g->d.h * g->d.h;
    return g->d.dtype == CS_F32 ? (double)(float)h2 : h2;
}

cs_status check_tmp(const cs_grid_s* g, const void* tmp, bool* pairs = nullptr)
{
    if (tmp == g->u || tmp == g->b) { set_error("u_tmp must be a separate array"); return CS_EINVAL; }
    size_t before = 0, after = 0;
    cs_status st = check_device_range(tmp, (size_t)g->span * g->elem, g->elem, "u_tmp", &before, &after);
    if (st == CS_OK && pairs) *pairs = pair_layout(g->geo, g->d.dim, tmp, g->elem, before, after);
    return st;
}

}  // namespace

cs_status check_device_range_pub(const void* p, size_t bytes, size_t align, const char* name)
{
    return check_device_range(p, bytes, align, name);
}

cs_status validate_desc_pub(const cs_grid_desc* d)
{
    return validate_desc(d);
}

int64_t span_of_pub(const cs_grid_desc& d)
{
    return span_of(d);
}

}  // namespace cs

using namespace cs;

extern "C" {

const char* cs_last_error(void) { return g_err; }

cs_status cs_grid_create(const cs_grid_desc* desc, void* u, const void* b, cs_grid* out)
{
    g_err[0] = 0;
    if (!out) { set_error("out is NULL"); return CS_EINVAL; }
    *out = nullptr;
    cs_status st = validate_desc(desc);
    if (st != CS_OK) return st;
    const size_t elem = desc->dtype == CS_F64 ? 8 : 4;
    const int64_t span = span_of(*desc);
    size_t u_before = 0, u_after = 0;
    if ((st = check_device_range(u, (size_t)span * elem, elem, "u", &u_before, &u_after)) != CS_OK) return st;
    if ((st = check_device_range(b, (size_t)span * elem, elem, "b")) != CS_OK) return st;
    if (u == b) { set_error("u and b must be separate arrays"); return CS_EINVAL; }
    cs_grid_s* g = new (std::nothrow) cs_grid_s();
    if (!g) { set_error("out of host memory"); return CS_ENOMEM; }
    g->d = *desc;
    if (g->d.dim == 2) { g->d.n[2] = 1; g->d.stride[2] = 0; }
    g->geo.nx = g->d.n[0];
    g->geo.ny = g->d.n[1];
    g->geo.nz = g->d.dim == 3 ? g->d.n[2] : 1;
    g->geo.sy = g->d.stride[1];
    g->geo.sz = g->d.dim == 3 ? g->d.stride[2] : 0;
    g->geo.parity = g->d.parity;
    g->u = u;
    g->b = b;
    g->elem = elem;
    g->span = span;
    g->pair_loads = pair_layout(g->geo, g->d.dim, u, elem, u_before, u_after);
    hipError_t e = hipGetDevice(&g->device);
    if (e != hipSuccess) { delete g; return hip_fail(e, "hipGetDevice"); }
    e = hipMalloc((void**)&g->partials, sizeof(Partial) * kMaxResidualBlocks);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        delete g;
        set_error("hipMalloc of the reduction scratch failed: %s", hipGetErrorString(e));
        return CS_ENOMEM;
    }
    // barrier words of the persistent sweeps, then one counter per tile of
    // the dependency-driven sweep
    int64_t tnx = 0, tny = 0, tnz = 0;
    dep_tile_counts(g->geo, g->d.dim, &tnx, &tny, &tnz);
    const size_t words = 4 + (size_t)(tnx * tny * tnz);
    e = hipMalloc((void**)&g->bar, words * sizeof(unsigned));
    if (e == hipSuccess) e = hipMemset(g->bar, 0, words * sizeof(unsigned));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(g->partials);
        if (g->bar) (void)hipFree(g->bar);
        delete g;
        set_error("allocation of the barrier words failed: %s", hipGetErrorString(e));
        return CS_ENOMEM;
    }
    *out = g;
    return CS_OK;
}

cs_status cs_grid_destroy(cs_grid g)
{
    if (!g) return CS_OK;
    hipError_t e = hipFree(g->partials);
    const hipError_t e2 = hipFree(g->bar);
    if (e == hipSuccess) e = e2;
    if (g->nd_nodes) {
        const hipError_t e3 = hipFree(g->nd_nodes);
        if (e == hipSuccess) e = e3;
    }
    delete g->nd_stage_off;
    delete g;
    if (e != hipSuccess) return hip_fail(e, "hipFree");
    return CS_OK;
}

cs_status cs_num_colours(cs_grid g, int32_t* out)
{
    if (!g || !out) { set_error("NULL argument"); return CS_EINVAL; }
    *out = g->d.stencil == CS_FD ? 2 : (1 << g->d.dim);
    return CS_OK;
}

// Sweeps per pass of cs_gs_sweeps (with a work array) and whether
// cs_jacobi_sweeps pairs its sweeps, on this grid under its pass mode.  2D
// grids take up to fused2d_max_sweeps sweeps per launch (an LDS-resident
// tile), 3D red-black grids two.
// Schedules of small 3D grids in the automatic mode, from sweep times on
// MI355X (FP64, us per sweep, fused pass / one launch per colour / one
// workgroup): 7^3 7-point 12.1 / 7.7 / 3.4, 15^3 22.0 / 7.6 / 5.3, 23^3 -- /
// -- / 14.4, 63^3 17.4 / 7.6 / 273; 27-point 7^3 14.0 / 23.5 / 6.4, 15^3
// 25.0 / 23.0 / 12.6, 63^3 21.4 / 23.0 / 514; at 127^3 the fused pass is
// level with the colour launches (7-point) or ahead (27-point).  Up to 16^3
// points every sweep runs in one workgroup; 7-point grids up to ~100^3 run one
// launch per colour, in place.
// Automatic schedule of the 3D sweeps, per [stencil][dtype] (process-wide,
// set by cs_grid_schedule_policy and the autotuner): all sweeps in one
// workgroup up to block_max points, one launch per colour up to colour_max
// points, else fused passes, two sweeps per pass from two_min points on where
// the double sweep is built (two_min < 0: where the grid fills the device).
// The defaults are measured at 7^3 .. 256^3 (FP64): the one-workgroup
// schedule wins up to about 16^3, the 7-point colour launches up to about
// 100^3, the 27-point double sweep nowhere.
struct SchedPolicy {
    int64_t block_max, colour_max, two_min;
};
constexpr int64_t kNever = INT64_MAX;
constexpr SchedPolicy kSchedDefault[2] = {{4096, 1100000, -1}, {4096, 0, kNever}};
SchedPolicy g_sched[2][2] = {{kSchedDefault[0], kSchedDefault[0]}, {kSchedDefault[1], kSchedDefault[1]}};

static int64_t points_of(cs_grid g)
{
    return g->geo.nx * g->geo.ny * g->geo.nz;
}

static const SchedPolicy& sched_of(cs_grid g)
{
    return g_sched[g->d.stencil][g->d.dtype];
}

static bool block_sweeps_pay(cs_grid g)
{
    return g->d.dim == 3 && points_of(g) <= sched_of(g).block_max;
}

static bool colour_launches_pay(cs_grid g)
{
    return g->d.dim == 3 && points_of(g) <= sched_of(g).colour_max;
}

static int gs_per_pass(cs_grid g)
{
    const int dt = g->d.dtype, dim = g->d.dim, sten = g->d.stencil;
    if (g->pass_mode == CS_PASS_ONE || !fused_supported(dt, dim, sten, g->geo)) return 1;
    if (dim == 2) return fused2d_max_sweeps(sten);
    if (g->pass_mode == CS_PASS_TWO) return fused_two_available(dt, dim, sten, g->geo) ? 2 : 1;
    const int64_t two_min = sched_of(g).two_min;
    if (two_min < 0) return fused_two_preferred(dt, dim, sten, g->geo) ? 2 : 1;
    return fused_two_available(dt, dim, sten, g->geo) && points_of(g) >= two_min ? 2 : 1;
}

static int jacobi_per_pass(cs_grid g)
{
    if (g->pass_mode == CS_PASS_ONE) return 1;
    if (g->d.dim == 2) return jacobi2d_max_sweeps(g->geo);
    return jacobi3_two_supported(g->d.stencil, g->geo) ? 2 : 1;
}

cs_status cs_grid_schedule_policy(int32_t stencil, int32_t dtype, int64_t block_max, int64_t colour_max,
                                  int64_t two_min)
{
    if ((stencil != CS_FD && stencil != CS_Q1) || (dtype != CS_F64 && dtype != CS_F32)) {
        set_error("bad stencil or dtype");
        return CS_EINVAL;
    }
    const SchedPolicy& d = kSchedDefault[stencil];
    SchedPolicy& p = g_sched[stencil][dtype];
    p.block_max = block_max >= 0 ? block_max : d.block_max;
    p.colour_max = colour_max >= 0 ? colour_max : d.colour_max;
    p.two_min = two_min >= 0 ? two_min : d.two_min;
    return CS_OK;
}

cs_status cs_grid_set_pass_mode(cs_grid g, int32_t mode)
{
    cs_status st = check_grid(g);
    if (st != CS_OK) return st;
    if (mode != CS_PASS_AUTO && mode != CS_PASS_ONE && mode != CS_PASS_TWO) {
        set_error("pass mode must be CS_PASS_AUTO, CS_PASS_ONE or CS_PASS_TWO");
        return CS_EINVAL;
    }
    g->pass_mode = mode;
    return CS_OK;
}

cs_status cs_sweeps_per_pass(cs_grid g, int32_t jacobi, int32_t* out)
{
    cs_status st = check_grid(g);
    if (st != CS_OK) return st;
    if (!out) { set_error("out is NULL"); return CS_EINVAL; }
    if (jacobi != 0 && jacobi != 1) { set_error("jacobi must be 0 or 1"); return CS_EINVAL; }
    *out = jacobi ? jacobi_per_pass(g) : gs_per_pass(g);
    return CS_OK;
}

cs_status cs_gs_fused(cs_grid g, int32_t* out)
{
    if (!g || !out) { set_error("NULL argument"); return CS_EINVAL; }
    *out = fused_supported(g->d.dtype, g->d.dim, g->d.stencil, g->geo) ? 1 : 0;
    return CS_OK;
}

cs_status cs_colour_pass(cs_grid g, int32_t colour, void* stream)
{
    cs_status st = check_grid(g);
    if (st != CS_OK) return st;
    const int nc = g->d.stencil == CS_FD ? 2 : (1 << g->d.dim);
    if (colour < 0 || colour >= nc) { set_error("colour %d outside [0, %d)", colour, nc); return CS_EINVAL; }
    return launch_colour_pass(g->d.dtype, g->d.dim, g->d.stencil, g->geo, g->u, g->b, h2_of(g),
                              colour, (hipStream_t)stream);
}

cs_status cs_gs_sweeps(cs_grid g, int32_t nsweeps, void* u_tmp, void* stream)
{
    cs_status st = check_grid(g);
    if (st != CS_OK) return st;
    if (nsweeps < 0) { set_error("nsweeps must be >= 0"); return CS_EINVAL; }
    if (nsweeps == 0) return CS_OK;
    hipStream_t s = (hipStream_t)stream;
    const double h2 = h2_of(g);
    const int dt = g->d.dtype, dim = g->d.dim, sten = g->d.stencil;
    bool tmp_pairs = false;
    if (u_tmp) {
        if ((st = check_tmp(g, u_tmp, &tmp_pairs)) != CS_OK) return st;
    }
    const bool automatic = g->pass_mode == CS_PASS_AUTO;
    if (automatic && block_sweeps_pay(g))
        return launch_block_sweeps(dt, dim, sten, g->geo, g->u, g->b, h2, nsweeps, s);
    if (u_tmp && fused_supported(dt, dim, sten, g->geo) && !(automatic && colour_launches_pay(g))) {
        if ((st = launch_halo_copy(dt, dim, g->geo, g->u, u_tmp, s)) != CS_OK) return st;
        const void* src = g->u;
        void* dst = u_tmp;
        const int per = gs_per_pass(g);
        // 3D: double sweeps first, then single ones.  An odd number of passes
        // leaves the iterate in u_tmp and costs a copy back; in the automatic
        // mode one double sweep then runs as two single passes instead, which
        // is cheaper than the copy (at 256^3 FP64: 2 x 85 us against
        // 131 + 56 us).
        int32_t pairs = (dim == 3 && per == 2) ? nsweeps / 2 : 0;
        if (g->pass_mode == CS_PASS_AUTO && pairs > 0 && ((pairs + (nsweeps - 2 * pairs)) & 1)) --pairs;
        for (int32_t it = 0; it < nsweeps;) {
            if (dim == 2) {
                int sw = per;
                while (sw > nsweeps - it) sw >>= 1;  // 8, 4, 2, 1
                st = launch_fused2d(dt, sten, sw, g->geo, src, dst, g->b, h2, s);
                it += sw;
            } else if (it < 2 * pairs) {
                st = launch_fused_two(dt, dim, sten, g->geo, src, dst, g->b, h2, s);
                it += 2;
            } else {
                st = launch_fused_sweep(dt, dim, sten, g->geo, src, dst, g->b, h2, s,
                                        src == g->u ? g->pair_loads : tmp_pairs);
                it += 1;
            }
            if (st != CS_OK) return st;
            void* nsrc = dst;
            dst = (void*)src;
            src = nsrc;
        }
        if (src != g->u) return launch_interior_copy(dt, dim, g->geo, src, g->u, s);
        return CS_OK;
    }
    const int nc = sten == CS_FD ? 2 : (1 << dim);
    for (int32_t it = 0; it < nsweeps; ++it)
        for (int c = 0; c < nc; ++c)
            if ((st = launch_colour_pass(dt, dim, sten, g->geo, g->u, g->b, h2, c, s)) != CS_OK)
                return st;
    return CS_OK;
}

cs_status cs_fill_uniform(const cs_grid_desc* desc, void* a, uint64_t seed, void* stream)
{
    g_err[0] = 0;
    cs_status st = validate_desc(desc);
    if (st != CS_OK) return st;
    const size_t elem = desc->dtype == CS_F64 ? 8 : 4;
    if ((st = check_device_range(a, (size_t)span_of(*desc) * elem, elem, "a")) != CS_OK) return st;
    Geo geo;
    geo.nx = desc->n[0];
    geo.ny = desc->n[1];
    geo.nz = desc->dim == 3 ? desc->n[2] : 1;
    geo.sy = desc->stride[1];
    geo.sz = desc->dim == 3 ? desc->stride[2] : 0;
    geo.parity = desc->parity;
    return launch_fill_uniform(desc->dtype, desc->dim, geo, a, seed, (hipStream_t)stream);
}

cs_status cs_apply(cs_grid g, void* y, int32_t cellwise, void* stream)
{
    cs_status st = check_grid(g);
    if (st != CS_OK) return st;
    if (!y) { set_error("y is NULL"); return CS_EINVAL; }
    if ((st = check_tmp(g, y)) != CS_OK) return st;
    if (cellwise != 0 && cellwise != 1) { set_error("cellwise must be 0 or 1"); return CS_EINVAL; }
    if (cellwise && g->d.stencil != CS_Q1) {
        set_error("the cell-wise form exists for the d-linear stencils only");
        return CS_EINVAL;
    }
    return launch_apply(g->d.dtype, g->d.dim, g->d.stencil, g->geo, g->u, y, h2_of(g), cellwise,
                        (hipStream_t)stream);
}

cs_status cs_gs_sweeps_sync(cs_grid g, int32_t nsweeps, void* stream)
{
    cs_status st = check_grid(g);
    if (st != CS_OK) return st;
    if (nsweeps < 0) { set_error("nsweeps must be >= 0"); return CS_EINVAL; }
    if (nsweeps == 0) return CS_OK;
    return launch_sync_sweeps(g->d.dtype, g->d.dim, g->d.stencil, g->geo, g->u, g->b, h2_of(g),
                              nsweeps, g->bar, (hipStream_t)stream);
}

cs_status cs_gs_sweeps_dep(cs_grid g, int32_t nsweeps, void* stream)
{
    cs_status st = check_grid(g);
    if (st != CS_OK) return st;
    if (nsweeps < 0) { set_error("nsweeps must be >= 0"); return CS_EINVAL; }
    if (nsweeps == 0) return CS_OK;
    const int64_t phases = (int64_t)nsweeps * (g->d.stencil == CS_FD ? 2 : (1 << g->d.dim));
    if (phases >= ((int64_t)1 << 31)) { set_error("too many sweeps for the phase counters"); return CS_EINVAL; }
    return launch_dep_sweeps(g->d.dtype, g->d.dim, g->d.stencil, g->geo, g->u, g->b, h2_of(g),
                             nsweeps, g->bar, (hipStream_t)stream);
}

cs_status cs_gs_sweeps_nd(cs_grid g, int32_t nsweeps, int32_t leaf, void* stream)
{
    cs_status st = check_grid(g);
    if (st != CS_OK) return st;
    if (nsweeps < 0) { set_error("nsweeps must be >= 0"); return CS_EINVAL; }
    if (leaf < 1) { set_error("leaf must be >= 1"); return CS_EINVAL; }
    if (nsweeps == 0) return CS_OK;
    if (g->geo.nx >= (1LL << 30) || g->geo.ny >= (1LL << 30) || g->geo.nz >= (1LL << 30)) {
        set_error("nested dissection: sizes beyond 2^30");
        return CS_EUNSUPPORTED;
    }
    if (g->nd_leaf != leaf) {
        // building the tree allocates and copies synchronously, which a
        // stream under graph capture must not see
        hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
        hipError_t ce = hipStreamIsCapturing((hipStream_t)stream, &cap);
        if (ce != hipSuccess) return hip_fail(ce, "hipStreamIsCapturing");
        if (cap != hipStreamCaptureStatusNone) {
            set_error("nested dissection: the tree for leaf %d is not built; make one "
                      "uncaptured call with this leaf before capturing", leaf);
            return CS_EINVAL;
        }
        std::vector<NdNode> nodes;
        std::vector<int> off;
        if ((st = nd_tree(g->geo, g->d.dim, leaf, &nodes, &off)) != CS_OK) return st;
        if (g->nd_nodes) {
            hipError_t e = hipFree(g->nd_nodes);
            g->nd_nodes = nullptr;
            g->nd_leaf = 0;
            if (e != hipSuccess) return hip_fail(e, "hipFree");
        }
        hipError_t e = hipMalloc((void**)&g->nd_nodes, nodes.size() * sizeof(NdNode));
        if (e == hipSuccess)
            e = hipMemcpy(g->nd_nodes, nodes.data(), nodes.size() * sizeof(NdNode), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            if (g->nd_nodes) (void)hipFree(g->nd_nodes);
            g->nd_nodes = nullptr;
            set_error("allocation of the dissection tree failed: %s", hipGetErrorString(e));
            return CS_ENOMEM;
        }
        if (!g->nd_stage_off) {
            g->nd_stage_off = new (std::nothrow) std::vector<int>();
            if (!g->nd_stage_off) { set_error("out of host memory"); return CS_ENOMEM; }
        }
        *g->nd_stage_off = off;
        g->nd_leaf = leaf;
    }
    return launch_nd_sweeps(g->d.dtype, g->d.dim, g->d.stencil, g->geo, g->u, g->b, h2_of(g), nsweeps,
                            g->nd_nodes, g->nd_stage_off->data(), (int)g->nd_stage_off->size() - 1,
                            (hipStream_t)stream);
}

cs_status cs_gs_sync_failures(cs_grid g, int32_t* out, void* stream)
{
    cs_status st = check_grid(g);
    if (st != CS_OK) return st;
    if (!out) { set_error("out is NULL"); return CS_EINVAL; }
    unsigned words[4] = {0, 0, 0, 0};
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(words, g->bar, sizeof(words), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "reading the barrier words");
    *out = (int32_t)words[2];
    return CS_OK;
}

cs_status cs_gs_sweeps_lex(cs_grid g, int32_t nsweeps, void* stream)
{
    cs_status st = check_grid(g);
    if (st != CS_OK) return st;
    if (nsweeps < 0) { set_error("nsweeps must be >= 0"); return CS_EINVAL; }
    for (int32_t it = 0; it < nsweeps; ++it)
        if ((st = launch_lex_sweep(g->d.dtype, g->d.dim, g->d.stencil, g->geo, g->u, g->b, h2_of(g),
                                   (hipStream_t)stream)) != CS_OK)
            return st;
    return CS_OK;
}

cs_status cs_gs_sweeps_cost(cs_grid g, int32_t nsweeps, int32_t kmax, int32_t hetero, void* stream)
{
    cs_status st = check_grid(g);
    if (st != CS_OK) return st;
    if (nsweeps < 0) { set_error("nsweeps must be >= 0"); return CS_EINVAL; }
    if (kmax < 0 || kmax > 100000) { set_error("kmax %d outside [0, 100000]", kmax); return CS_EINVAL; }
    if (hetero != 0 && hetero != 1) { set_error("hetero must be 0 or 1"); return CS_EINVAL; }
    const int dt = g->d.dtype, dim = g->d.dim, sten = g->d.stencil;
    const Geo& geo = g->geo;
    StencilCost cost;
    cost.kmax = kmax;
    cost.hetero = hetero;
    cost.npts = geo.nx * geo.ny * geo.nz;
    cost.zero = 0.0;
    cost.a = 1.0 / 1024.0;
    cost.c = 1.0 / 128.0;
    const int nc = sten == CS_FD ? 2 : (1 << dim);
    for (int32_t it = 0; it < nsweeps; ++it)
        for (int c = 0; c < nc; ++c)
            if ((st = launch_colour_pass(dt, dim, sten, geo, g->u, g->b, h2_of(g), c,
                                         (hipStream_t)stream, &cost)) != CS_OK)
                return st;
    return CS_OK;
}

cs_status cs_jacobi_sweeps(cs_grid g, double omega, int32_t nsweeps, void* u_tmp, void* stream)
{
    cs_status st = check_grid(g);
    if (st != CS_OK) return st;
    if (nsweeps < 0) { set_error("nsweeps must be >= 0"); return CS_EINVAL; }
    if (!std::isfinite(omega)) { set_error("omega must be finite"); return CS_EINVAL; }
    if (!u_tmp) { set_error("Jacobi needs u_tmp"); return CS_EINVAL; }
    if ((st = check_tmp(g, u_tmp)) != CS_OK) return st;
    if (nsweeps == 0) return CS_OK;
    hipStream_t s = (hipStream_t)stream;
    const int dt = g->d.dtype, dim = g->d.dim, sten = g->d.stencil;
    if ((st = launch_halo_copy(dt, dim, g->geo, g->u, u_tmp, s)) != CS_OK) return st;
    const void* src = g->u;
    void* dst = u_tmp;
    const int per = jacobi_per_pass(g);
    for (int32_t it = 0; it < nsweeps;) {
        if (dim == 2 && per > 1) {
            int sw = per;
            while (sw > nsweeps - it) sw >>= 1;  // 8, 4, 2, 1
            st = launch_jacobi2d(dt, sten, sw, g->geo, src, dst, g->b, h2_of(g), omega, s);
            it += sw;
        } else if (per == 2 && nsweeps - it >= 2) {
            st = launch_jacobi3_two(dt, sten, g->geo, src, dst, g->b, h2_of(g), omega, s);
            it += 2;
        } else {
            st = launch_jacobi(dt, dim, sten, g->geo, src, dst, g->b, h2_of(g), omega, s);
            it += 1;
        }
        if (st != CS_OK) return st;
        void* nsrc = dst;
        dst = (void*)src;
        src = nsrc;
    }
    if (src != g->u) return launch_interior_copy(dt, dim, g->geo, src, g->u, s);
    return CS_OK;
}

cs_status cs_residual(cs_grid g, void* r, double* norms, void* stream)
{
    cs_status st = check_grid(g);
    if (st != CS_OK) return st;
    if (!norms && !r) { set_error("neither r nor norms given"); return CS_EINVAL; }
    if (norms && (st = check_device_range(norms, 3 * sizeof(double), sizeof(double), "norms")) != CS_OK)
        return st;
    if (r) {
        if (r == g->u || r == g->b) { set_error("r must be a separate array"); return CS_EINVAL; }
        if ((st = check_device_range(r, (size_t)g->span * g->elem, g->elem, "r")) != CS_OK) return st;
    }
    return launch_residual(g->d.dtype, g->d.dim, g->d.stencil, g->geo, g->u, g->b, r,
                           g->d.h * g->d.h, g->partials, norms, (hipStream_t)stream);
}

// A fine and a coarse grid of one multigrid hierarchy: same dim, stencil and
// dtype, fine n = 2 coarse n + 1 along every axis of the grid.
static cs_status check_mg_pair(cs_grid fine, cs_grid coarse)
{
    cs_status st = check_grid(fine);
    if (st != CS_OK) return st;
    if ((st = check_grid(coarse)) != CS_OK) return st;
    if (fine->d.dim != coarse->d.dim || fine->d.stencil != coarse->d.stencil ||
        fine->d.dtype != coarse->d.dtype) {
        set_error("multigrid grids differ in dim, stencil or dtype");
        return CS_EINVAL;
    }
    for (int a = 0; a < fine->d.dim; ++a)
        if (fine->d.n[a] != 2 * coarse->d.n[a] + 1) {
            set_error("fine n[%d] = %lld is not 2 * coarse n + 1 (coarse n = %lld)", a,
                      (long long)fine->d.n[a], (long long)coarse->d.n[a]);
            return CS_EINVAL;
        }
    if (fine->u == coarse->u || fine->u == coarse->b || (const void*)coarse->u == fine->b) {
        set_error("multigrid grids share an array");
        return CS_EINVAL;
    }
    return CS_OK;
}

cs_status cs_restrict(cs_grid fine, const void* r, cs_grid coarse, void* stream)
{
    cs_status st = check_mg_pair(fine, coarse);
    if (st != CS_OK) return st;
    if (r == coarse->u || r == coarse->b || r == fine->u) {
        set_error("r must be a separate array");
        return CS_EINVAL;
    }
    if ((st = check_device_range(r, (size_t)fine->span * fine->elem, fine->elem, "r")) != CS_OK)
        return st;
    return launch_restrict(fine->d.dtype, fine->d.dim, fine->geo, r, coarse->geo,
                           const_cast<void*>(coarse->b), coarse->u, (hipStream_t)stream);
}

cs_status cs_prolong_add(cs_grid coarse, cs_grid fine, void* stream)
{
    cs_status st = check_mg_pair(fine, coarse);
    if (st != CS_OK) return st;
    return launch_prolong_add(fine->d.dtype, fine->d.dim, coarse->geo, coarse->u, fine->geo,
                              fine->u, (hipStream_t)stream);
}

static cs_status check_ir_pair(cs_grid g64, cs_grid g32, double scale)
{
    cs_status st = check_grid(g64);
    if (st != CS_OK) return st;
    if ((st = check_grid(g32)) != CS_OK) return st;
    if (g64->d.dtype != CS_F64 || g32->d.dtype != CS_F32) {
        set_error("refinement needs an FP64 grid and an FP32 grid");
        return CS_EINVAL;
    }
    if (g64->d.dim != g32->d.dim || g64->d.stencil != g32->d.stencil ||
        g64->d.parity != g32->d.parity || g64->d.h != g32->d.h || g64->d.n[0] != g32->d.n[0] ||
        g64->d.n[1] != g32->d.n[1] || g64->d.n[2] != g32->d.n[2]) {
        set_error("refinement grids differ in dim, stencil, parity, n or h");
        return CS_EINVAL;
    }
    int ex = 0;
    if (!(scale > 0.0) || !std::isfinite(scale) || std::frexp(scale, &ex) != 0.5) {
        set_error("scale must be a positive power of two");
        return CS_EINVAL;
    }
    return CS_OK;
}

cs_status cs_ir_residual(cs_grid g64, cs_grid g32, double scale, double* norms, void* stream)
{
    cs_status st = check_ir_pair(g64, g32, scale);
    if (st != CS_OK) return st;
    if ((st = check_device_range(norms, 3 * sizeof(double), sizeof(double), "norms")) != CS_OK)
        return st;
    return launch_ir_residual(g64->d.dim, g64->d.stencil, g64->geo, g64->u, g64->b,
                              g64->d.h * g64->d.h, 1.0 / scale, g32->geo, (void*)g32->b, g32->u,
                              g64->partials, norms, (hipStream_t)stream);
}

cs_status cs_ir_update(cs_grid g64, cs_grid g32, double scale, void* stream)
{
    cs_status st = check_ir_pair(g64, g32, scale);
    if (st != CS_OK) return st;
    return launch_ir_update(g64->d.dim, g64->geo, g64->u, g32->geo, g32->u, scale,
                            (hipStream_t)stream);
}

}  // extern "C"
