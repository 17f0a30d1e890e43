// C ABI of the batched patches: validation, grouping, device tables, the
// per-sweep launches and the batched refinement steps.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <new>
#include <vector>

#include "cs_batch.h"

using namespace cs;

namespace {

struct Group {
    int dtype = 0, stencil = 0, variant = 0;
    int tier = 0;        // LDS-resident tier (1, 2), plane streaming (3, or 5 in its small
                         // form), colour passes (4), or 0 for the tile kernels
    bool pairs = false;  // two sweeps per launch
    std::vector<BatchPatch> host;
    BatchPatch* dev = nullptr;
    int64_t items = 0, res_items = 0, halo_items = 0, partial_base = 0;
};

// [stencil][dtype]: below these totals a tiled group runs faster as colour
// passes (measured on groups of the largest patches of a request stream: the
// colour passes win for one such patch, about 1M points, and lose from two
// on, except FP32 27-point groups, where they win up to about 6M points).
constexpr int64_t kColourMax[2][2] = {{(int64_t)5 << 18, (int64_t)6 << 18},
                                      {(int64_t)4 << 18, (int64_t)16 << 18}};

// [stencil][dtype].  By default every tiled patch takes the large tiles: on
// patches of arbitrary shape (the tiled ones, now that small patches are
// resident or streamed) they sweep fastest despite their ragged edge tiles.
int g_small_max[2][2] = {{0, 0}, {0, 0}};
int g_mid_max[2][2] = {{0, 0}, {0, 0}};
int g_pair_large[2][2] = {{1, 1}, {1, 1}};  // pair the sweeps of the large tile class
// Tiled groups of fewer interior points than this are swept by colour passes
// instead (a small group gives the tile kernels too few work items).
int64_t g_colour_max[2][2] = {{kColourMax[0][0], kColourMax[0][1]}, {kColourMax[1][0], kColourMax[1][1]}};
int g_resident[2][2] = {{3, 3}, {3, 3}};    // bit 0: whole patches in LDS; bit 1: plane streaming
                                            // for large classes; bit 2: plane streaming always

int pick_variant(int stencil, int dtype, int64_t nx)
{
    if (nx <= g_small_max[stencil][dtype]) return 0;
    if (nx <= g_mid_max[stencil][dtype]) return 1;
    return 2;
}

int64_t span_of3(const cs_grid_desc& d)
{
    return (d.n[2] + 1) * d.stride[2] + (d.n[1] + 1) * d.stride[1] + d.n[0] + 2;
}

// Plane streaming gives each patch one workgroup for all its sweeps: it pays
// only when a group holds at least one such patch for every compute unit;
// fewer would leave most of the device idle while the tile kernels could
// spread the same patches over all of it.
int planes_min_patches()
{
    static std::atomic<int> cu[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
        (void)hipGetLastError();
        return 256;
    }
    int n = cu[dev].load(std::memory_order_relaxed);
    if (n < 1) {
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1) {
            (void)hipGetLastError();
            n = 256;
        }
        cu[dev].store(n, std::memory_order_relaxed);
    }
    return n;
}

// Host plan of a batch: its groups (tables not yet on the device), the sweeps
// per pass of every patch in the caller's order, the residual partials it
// needs, the number of norm rows, and every patch in the caller's order.
struct Plan {
    std::vector<Group> groups;
    std::vector<int> per_pass;
    std::vector<BatchPatch> by_index;
    int64_t partials = 0;
    int rows = 0;
};

cs_status plan_batch(const cs_grid_desc* descs, void* const* u, const void* const* b,
                     void* const* tmp, const int32_t* rows, int32_t count, Plan* pl)
{
    if (count < 0) { set_error("count must be >= 0"); return CS_EINVAL; }
    if (count > 0 && (!descs || !u || !b || !tmp)) { set_error("NULL array"); return CS_EINVAL; }
    std::vector<int32_t> seen;
    // plane-streaming candidates per [stencil][dtype]; a class with fewer
    // than planes_min_patches() of them keeps the tile kernels
    int planes_cand[2][2] = {{0, 0}, {0, 0}};
    for (int32_t i = 0; i < count; ++i) {
        const cs_grid_desc& d = descs[i];
        if (validate_desc_pub(&d) != CS_OK || d.dim != 3) continue;  // reported below
        Geo g{};
        g.nx = d.n[0];
        g.ny = d.n[1];
        g.nz = d.n[2];
        const int pol = g_resident[d.stencil][d.dtype];
        if ((pol & 6) && !((pol & 1) && batch_resident_tier(d.dtype, d.stencil, g)) &&
            batch_planes_fits(d.dtype, d.stencil, g))
            ++planes_cand[d.stencil][d.dtype];
    }
    const int planes_min = planes_min_patches();
    std::vector<int> gidx;  // group of each patch, caller's order
    for (int32_t i = 0; i < count; ++i) {
        const cs_grid_desc& d = descs[i];
        cs_status st = validate_desc_pub(&d);
        if (st != CS_OK) return st;
        if (d.dim != 3) { set_error("patch %d: batches hold 3D patches", i); return CS_EUNSUPPORTED; }
        if ((d.n[1] + 2) * d.stride[1] >= ((int64_t)1 << 31)) {
            set_error("patch %d: plane too large for 32-bit offsets", i);
            return CS_EUNSUPPORTED;
        }
        const size_t elem = d.dtype == CS_F64 ? 8 : 4;
        const size_t bytes = (size_t)span_of3(d) * elem;
        if ((st = check_device_range_pub(u[i], bytes, elem, "patch u")) != CS_OK ||
            (st = check_device_range_pub(b[i], bytes, elem, "patch b")) != CS_OK ||
            (st = check_device_range_pub(tmp[i], bytes, elem, "patch tmp")) != CS_OK)
            return st;
        if (u[i] == tmp[i] || u[i] == b[i] || tmp[i] == b[i]) {
            set_error("patch %d: u, b and tmp must be separate arrays", i);
            return CS_EINVAL;
        }
        const int32_t row = rows ? rows[i] : i;
        if (row < 0 || row >= (1 << 30)) { set_error("patch %d: norm row %d out of range", i, row); return CS_EINVAL; }
        seen.push_back(row);
        BatchPatch p{};
        p.g.nx = d.n[0];
        p.g.ny = d.n[1];
        p.g.nz = d.n[2];
        p.g.sy = d.stride[1];
        p.g.sz = d.stride[2];
        p.g.parity = d.parity;
        p.u = (CS_GLOBAL void*)u[i];
        p.tmp = (CS_GLOBAL void*)tmp[i];
        p.b = (const CS_GLOBAL void*)b[i];
        p.hh = d.h * d.h;
        p.h2 = d.dtype == CS_F32 ? (double)(float)p.hh : p.hh;
        p.index = row;
        p.stencil = d.stencil;
        p.dtype = d.dtype;
        const int pol = g_resident[d.stencil][d.dtype];
        int tier = (pol & 1) ? batch_resident_tier(d.dtype, d.stencil, p.g) : 0;
        if (!tier && ((pol & 4) || ((pol & 2) && planes_cand[d.stencil][d.dtype] >= planes_min)) &&
            batch_planes_fits(d.dtype, d.stencil, p.g))
            tier = batch_planes_small(d.dtype, d.stencil, p.g) ? 5 : 3;
        const int variant = tier ? 0 : pick_variant(d.stencil, d.dtype, d.n[0]);
        const bool pairs = !tier && batch_variant_pairs(d.stencil, variant) && g_pair_large[d.stencil][d.dtype];
        int tx = 0, ty = 0;
        batch_variant_tile(d.stencil, variant, &tx, &ty);
        p.tiles_x = (int)((d.n[0] + tx - 1) / tx);
        p.tiles_y = (int)((d.n[1] + ty - 1) / ty);
        p.chunks = 1;  // set below, once the batch's total tile count is known
        p.res_items = (int)batch_residual_items(p.g);
        int k = -1;
        for (size_t j = 0; j < pl->groups.size(); ++j)
            if (pl->groups[j].dtype == d.dtype && pl->groups[j].stencil == d.stencil &&
                pl->groups[j].variant == variant && pl->groups[j].pairs == pairs &&
                pl->groups[j].tier == tier)
                k = (int)j;
        if (k < 0) {
            Group gr;
            gr.dtype = d.dtype;
            gr.stencil = d.stencil;
            gr.variant = variant;
            gr.tier = tier;
            gr.pairs = pairs;
            pl->groups.push_back(gr);
            k = (int)pl->groups.size() - 1;
        }
        pl->groups[k].host.push_back(p);
        gidx.push_back(k);
        pl->by_index.push_back(p);
        pl->per_pass.push_back(tier == 3 || tier == 5 ? batch_planes_sweeps(d.dtype, d.stencil, p.g)
                               : (tier ? 0 : (pairs ? 2 : 1)));
        pl->rows = std::max(pl->rows, row + 1);
    }
    std::sort(seen.begin(), seen.end());
    if (std::adjacent_find(seen.begin(), seen.end()) != seen.end()) {
        set_error("two patches share a norm row");
        return CS_EINVAL;
    }
    // small tiled groups go to the colour passes (same iterate, in place)
    for (size_t j = 0; j < pl->groups.size(); ++j) {
        Group& gr = pl->groups[j];
        if (gr.tier) continue;
        int64_t pts = 0;
        for (auto& p : gr.host) pts += p.g.nx * p.g.ny * p.g.nz;
        if (pts >= g_colour_max[gr.stencil][gr.dtype]) continue;
        gr.tier = 4;
        gr.pairs = false;
        for (size_t i = 0; i < gidx.size(); ++i)
            if (gidx[i] == (int)j) pl->per_pass[i] = 1;
    }
    // z chunks: enough work items to fill the GPU (about 2048) when the batch
    // holds few patches, never chunks thinner than 8 planes (16 for the tile
    // class that also runs double sweeps).  The split does not change any
    // value: every point is computed the same way in any tile.
    int64_t total_tiles = 0;
    for (auto& gr : pl->groups)
        if (!gr.tier)
            for (auto& p : gr.host) total_tiles += (int64_t)p.tiles_x * p.tiles_y;
    const int64_t want = total_tiles > 0 ? (2048 + total_tiles - 1) / total_tiles : 1;
    for (auto& gr : pl->groups) {
        const int depth = gr.pairs ? 16 : 8;
        for (auto& p : gr.host)
            p.chunks = (int)std::max<int64_t>(1, std::min<int64_t>(want, p.g.nz / depth));
    }
    int64_t partial_total = 0;
    for (auto& gr : pl->groups) {
        std::stable_sort(gr.host.begin(), gr.host.end(), [](const BatchPatch& a, const BatchPatch& c) {
            return a.g.nx * a.g.ny * a.g.nz > c.g.nx * c.g.ny * c.g.nz;
        });
        int64_t it = 0, rit = 0, hit = 0;
        for (auto& p : gr.host) {
            p.halo_begin = hit;
            hit += p.g.nz + 2;
            p.item_begin = it;
            it += gr.tier == 4 ? batch_colour_items(gr.stencil, p.g)
                               : (gr.tier ? 1 : (int64_t)p.tiles_x * p.tiles_y * p.chunks);
            p.res_begin = rit;
            rit += p.res_items;
        }
        if (it > 0x7fffffff || rit > 0x7fffffff || hit > 0x7fffffff) {
            set_error("batch too large");
            return CS_EUNSUPPORTED;
        }
        gr.items = it;
        gr.res_items = rit;
        gr.halo_items = hit;
        gr.partial_base = partial_total;
        partial_total += rit;
    }
    pl->partials = partial_total;
    return CS_OK;
}

}  // namespace

// A batch owns a device table arena of `capacity` patches, a partials arena,
// two pinned host staging buffers for each table and the events of the
// copies out of them; the tables of an assignment are written into a staging
// buffer and copied asynchronously, so reassigning allocates nothing.
struct cs_batch_s {
    int count = 0;
    int device = 0;
    int capacity = 0;
    int rows = 0;                 // norm rows in use (largest row + 1)
    int64_t partial_cap = 0;
    std::vector<Group> groups;
    std::vector<int> per_pass;    // sweeps per launch of each patch (caller's order)
    std::vector<BatchPatch> by_index;
    BatchPatch* arena = nullptr;
    Partial* partials = nullptr;
    BatchPatch* stage[2] = {nullptr, nullptr};
    hipEvent_t staged[2] = {nullptr, nullptr};
    int next = 0;
    // refinement pairing (cs_batch_ir_attach): FP64 iterate and right-hand
    // side of each patch of this (FP32) batch
    IrPatch* ir_arena = nullptr;
    IrPatch* ir_stage[2] = {nullptr, nullptr};
    hipEvent_t ir_ev[2] = {nullptr, nullptr};
    int ir_next = 0;
    bool ir_ok = false;
    int64_t ir_items = 0;
};

static void free_batch(cs_batch_s* bt)
{
    if (!bt) return;
    if (bt->arena) (void)hipFree(bt->arena);
    if (bt->partials) (void)hipFree(bt->partials);
    if (bt->ir_arena) (void)hipFree(bt->ir_arena);
    for (int i = 0; i < 2; ++i) {
        if (bt->stage[i]) (void)hipHostFree(bt->stage[i]);
        if (bt->ir_stage[i]) (void)hipHostFree(bt->ir_stage[i]);
        if (bt->staged[i]) (void)hipEventDestroy(bt->staged[i]);
        if (bt->ir_ev[i]) (void)hipEventDestroy(bt->ir_ev[i]);
    }
    delete bt;
}

static cs_status alloc_batch(int capacity, int64_t partial_cap, cs_batch_s** out)
{
    *out = nullptr;
    cs_batch_s* bt = new (std::nothrow) cs_batch_s();
    if (!bt) { set_error("out of host memory"); return CS_ENOMEM; }
    hipError_t e = hipGetDevice(&bt->device);
    if (e != hipSuccess) { free_batch(bt); return hip_fail(e, "hipGetDevice"); }
    bt->capacity = capacity;
    bt->partial_cap = partial_cap;
    const size_t cap = (size_t)std::max(capacity, 1);
    e = hipMalloc((void**)&bt->arena, sizeof(BatchPatch) * cap);
    if (e == hipSuccess) e = hipMalloc((void**)&bt->partials, sizeof(Partial) * (size_t)std::max<int64_t>(partial_cap, 1));
    if (e == hipSuccess) e = hipMalloc((void**)&bt->ir_arena, sizeof(IrPatch) * cap);
    for (int i = 0; i < 2 && e == hipSuccess; ++i) {
        e = hipHostMalloc((void**)&bt->stage[i], sizeof(BatchPatch) * cap, hipHostMallocDefault);
        if (e == hipSuccess) e = hipHostMalloc((void**)&bt->ir_stage[i], sizeof(IrPatch) * cap, hipHostMallocDefault);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&bt->staged[i], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&bt->ir_ev[i], hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        free_batch(bt);
        set_error("allocation of the batch tables failed: %s", hipGetErrorString(e));
        return CS_ENOMEM;
    }
    *out = bt;
    return CS_OK;
}

// Take over a plan: its tables go through the next staging buffer (once the
// copy that last used it has run) into the arena, asynchronously on s.
static cs_status install_plan(cs_batch_s* bt, Plan& pl, hipStream_t s)
{
    const int st_i = bt->next;
    hipError_t e = hipEventSynchronize(bt->staged[st_i]);
    if (e != hipSuccess) return hip_fail(e, "waiting for a staging buffer");
    size_t off = 0;
    for (auto& gr : pl.groups) {
        std::copy(gr.host.begin(), gr.host.end(), bt->stage[st_i] + off);
        gr.dev = bt->arena + off;
        off += gr.host.size();
    }
    if (off > 0) {
        e = hipMemcpyAsync(bt->arena, bt->stage[st_i], sizeof(BatchPatch) * off, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipEventRecord(bt->staged[st_i], s);
        if (e != hipSuccess) return hip_fail(e, "patch table upload");
    }
    bt->next ^= 1;
    bt->groups.swap(pl.groups);
    bt->per_pass.swap(pl.per_pass);
    bt->by_index.swap(pl.by_index);
    bt->count = (int)bt->per_pass.size();
    bt->rows = pl.rows;
    bt->ir_ok = false;
    return CS_OK;
}

extern "C" {

cs_status cs_batch_tile_policy(int32_t stencil, int32_t dtype, int32_t small_max, int32_t mid_max)
{
    if ((stencil != CS_FD && stencil != CS_Q1) || (dtype != CS_F64 && dtype != CS_F32) ||
        small_max < 0 || small_max > mid_max) {
        set_error("bad tile policy");
        return CS_EINVAL;
    }
    g_small_max[stencil][dtype] = small_max;
    g_mid_max[stencil][dtype] = mid_max;
    return CS_OK;
}

cs_status cs_batch_pass_policy(int32_t stencil, int32_t dtype, int32_t pair_large)
{
    if ((stencil != CS_FD && stencil != CS_Q1) || (dtype != CS_F64 && dtype != CS_F32) ||
        (pair_large != 0 && pair_large != 1)) {
        set_error("bad pass policy");
        return CS_EINVAL;
    }
    g_pair_large[stencil][dtype] = pair_large;
    return CS_OK;
}

cs_status cs_batch_colour_policy(int32_t stencil, int32_t dtype, int64_t max_points)
{
    if ((stencil != CS_FD && stencil != CS_Q1) || (dtype != CS_F64 && dtype != CS_F32) || max_points < -1) {
        set_error("bad colour policy");
        return CS_EINVAL;
    }
    g_colour_max[stencil][dtype] = max_points >= 0 ? max_points : kColourMax[stencil][dtype];
    return CS_OK;
}

cs_status cs_batch_resident_policy(int32_t stencil, int32_t dtype, int32_t enable)
{
    if ((stencil != CS_FD && stencil != CS_Q1) || (dtype != CS_F64 && dtype != CS_F32) ||
        enable < 0 || enable > 7) {
        set_error("bad resident policy");
        return CS_EINVAL;
    }
    g_resident[stencil][dtype] = enable;
    return CS_OK;
}

cs_status cs_batch_create(const cs_grid_desc* descs, void* const* u, const void* const* b,
                          void* const* tmp, int32_t count, cs_batch* out)
{
    if (!out) { set_error("out is NULL"); return CS_EINVAL; }
    *out = nullptr;
    if (count < 1 || !descs || !u || !b || !tmp) { set_error("empty batch or NULL array"); return CS_EINVAL; }
    Plan pl;
    cs_status st = plan_batch(descs, u, b, tmp, nullptr, count, &pl);
    if (st != CS_OK) return st;
    cs_batch_s* bt = nullptr;
    if ((st = alloc_batch(count, pl.partials, &bt)) != CS_OK) return st;
    if ((st = install_plan(bt, pl, nullptr)) != CS_OK) { free_batch(bt); return st; }
    hipError_t e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) { free_batch(bt); return hip_fail(e, "patch table upload"); }
    *out = bt;
    return CS_OK;
}

cs_status cs_batch_reserve(int32_t capacity, int64_t partials, cs_batch* out)
{
    if (!out) { set_error("out is NULL"); return CS_EINVAL; }
    *out = nullptr;
    if (capacity < 1 || capacity > (1 << 24) || partials < 1 || partials > ((int64_t)1 << 31)) {
        set_error("capacity must lie in [1, 2^24] and partials in [1, 2^31]");
        return CS_EINVAL;
    }
    cs_batch_s* bt = nullptr;
    cs_status st = alloc_batch(capacity, partials, &bt);
    if (st != CS_OK) return st;
    *out = bt;
    return CS_OK;
}

cs_status cs_batch_assign(cs_batch bt, const cs_grid_desc* descs, void* const* u, const void* const* b,
                          void* const* tmp, const int32_t* rows, int32_t count, void* stream)
{
    if (!bt) { set_error("batch is NULL"); return CS_EINVAL; }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != bt->device) {
        (void)hipGetLastError();
        set_error("batch belongs to device %d", bt->device);
        return CS_EINVAL;
    }
    if (count > bt->capacity) { set_error("%d patches exceed the reserved %d", count, bt->capacity); return CS_EINVAL; }
    Plan pl;
    cs_status st = plan_batch(descs, u, b, tmp, rows, count, &pl);
    if (st != CS_OK) return st;
    if (pl.partials > bt->partial_cap) {
        set_error("the patches need %lld residual partials, %lld reserved", (long long)pl.partials,
                  (long long)bt->partial_cap);
        return CS_EINVAL;
    }
    return install_plan(bt, pl, (hipStream_t)stream);
}

cs_status cs_batch_ir_attach(cs_batch bt, const cs_grid_desc* descs64, void* const* x,
                             const void* const* b, void* stream)
{
    if (!bt) { set_error("batch is NULL"); return CS_EINVAL; }
    bt->ir_ok = false;
    const int count = bt->count;
    if (count > 0 && (!descs64 || !x || !b)) { set_error("NULL array"); return CS_EINVAL; }
    const int st_i = bt->ir_next;
    hipError_t e = hipEventSynchronize(bt->ir_ev[st_i]);
    if (e != hipSuccess) return hip_fail(e, "waiting for a staging buffer");
    int64_t items = 0;
    for (int i = 0; i < count; ++i) {
        const BatchPatch& p = bt->by_index[(size_t)i];
        const cs_grid_desc& d = descs64[i];
        cs_status st = validate_desc_pub(&d);
        if (st != CS_OK) return st;
        if (d.dim != 3 || d.dtype != CS_F64 || p.dtype != CS_F32 || d.stencil != p.stencil ||
            d.n[0] != p.g.nx || d.n[1] != p.g.ny || d.n[2] != p.g.nz) {
            set_error("patch %d: the FP64 patch must match its FP32 patch (3D, n, stencil)", i);
            return CS_EINVAL;
        }
        const size_t bytes = (size_t)span_of3(d) * 8;
        if ((st = check_device_range_pub(x[i], bytes, 8, "patch x")) != CS_OK ||
            (st = check_device_range_pub(b[i], bytes, 8, "patch b")) != CS_OK)
            return st;
        if (x[i] == b[i] || x[i] == (const void*)p.u || x[i] == (const void*)p.b || x[i] == (const void*)p.tmp) {
            set_error("patch %d: x must be separate from b and the FP32 arrays", i);
            return CS_EINVAL;
        }
        IrPatch q{};
        q.g.nx = d.n[0];
        q.g.ny = d.n[1];
        q.g.nz = d.n[2];
        q.g.sy = d.stride[1];
        q.g.sz = d.stride[2];
        q.g.parity = d.parity;
        q.g2 = p.g;
        q.x = (CS_GLOBAL double*)x[i];
        q.b = (const CS_GLOBAL double*)b[i];
        q.e = (CS_GLOBAL float*)p.u;
        q.r32 = (CS_GLOBAL float*)p.b;
        q.hh = d.h * d.h;
        q.stencil = d.stencil;
        q.row = p.index;
        q.res_begin = items;
        q.res_items = p.res_items;
        items += p.res_items;
        bt->ir_stage[st_i][i] = q;
    }
    if (items > bt->partial_cap) { set_error("refinement residual needs more partials than reserved"); return CS_EINVAL; }
    if (count > 0) {
        e = hipMemcpyAsync(bt->ir_arena, bt->ir_stage[st_i], sizeof(IrPatch) * (size_t)count,
                           hipMemcpyHostToDevice, (hipStream_t)stream);
        if (e == hipSuccess) e = hipEventRecord(bt->ir_ev[st_i], (hipStream_t)stream);
        if (e != hipSuccess) return hip_fail(e, "refinement table upload");
    }
    bt->ir_next ^= 1;
    bt->ir_items = items;
    bt->ir_ok = true;
    return CS_OK;
}

cs_status cs_batch_ir_residual(cs_batch bt, double* scales, double* norms, void* stream)
{
    if (!bt) { set_error("batch is NULL"); return CS_EINVAL; }
    if (!bt->ir_ok) { set_error("no FP64 patches attached since the last assignment"); return CS_EINVAL; }
    if (bt->count == 0) return CS_OK;
    cs_status st = check_device_range_pub(norms, sizeof(double) * 3 * (size_t)bt->rows, sizeof(double), "norms");
    if (st == CS_OK) st = check_device_range_pub(scales, sizeof(double) * (size_t)bt->rows, sizeof(double), "scales");
    if (st != CS_OK) return st;
    return launch_batch_ir_residual(bt->ir_arena, bt->count, bt->ir_items, bt->partials, scales,
                                    norms, (hipStream_t)stream);
}

cs_status cs_batch_ir_update(cs_batch bt, const double* scales, void* stream)
{
    if (!bt) { set_error("batch is NULL"); return CS_EINVAL; }
    if (!bt->ir_ok) { set_error("no FP64 patches attached since the last assignment"); return CS_EINVAL; }
    if (bt->count == 0) return CS_OK;
    cs_status st = check_device_range_pub(scales, sizeof(double) * (size_t)bt->rows, sizeof(double), "scales");
    if (st != CS_OK) return st;
    return launch_batch_ir_update(bt->ir_arena, bt->count, bt->ir_items, scales, (hipStream_t)stream);
}

cs_status cs_batch_destroy(cs_batch bt)
{
    free_batch(bt);
    return CS_OK;
}

cs_status cs_batch_gs_sweeps(cs_batch bt, int32_t nsweeps, void* stream)
{
    if (!bt) { set_error("batch is NULL"); return CS_EINVAL; }
    if (nsweeps < 0) { set_error("nsweeps must be >= 0"); return CS_EINVAL; }
    if (nsweeps == 0) return CS_OK;
    hipStream_t s = (hipStream_t)stream;
    cs_status st;
    // LDS-resident and plane-streaming groups: every sweep in one launch;
    // colour-pass groups: one launch per colour phase; all in place in u
    for (auto& gr : bt->groups) {
        if (!gr.tier) continue;
        const int n = (int)gr.host.size();
        if (gr.tier == 4)
            st = launch_batch_colour(gr.dtype, gr.stencil, gr.dev, n, gr.items, nsweeps, s);
        else if (gr.tier == 3 || gr.tier == 5)
            st = launch_batch_planes(gr.dtype, gr.stencil, gr.dev, n, nsweeps, s, gr.tier == 5);
        else
            st = launch_batch_resident(gr.dtype, gr.stencil, gr.tier, gr.dev, n, nsweeps, s);
        if (st != CS_OK) return st;
    }
    for (auto& gr : bt->groups)
        if (!gr.tier && (st = launch_batch_halo(gr.dtype, gr.dev, (int)gr.host.size(), gr.halo_items, s)) != CS_OK)
            return st;
    // Each launch reads u (phase 0) or tmp (phase 1) and writes the other; a
    // group whose sweeps run two per launch flips less often, so the copy back
    // into u is decided per group.
    std::vector<int> phase(bt->groups.size(), 0);
    for (int32_t it = 0; it < nsweeps;) {
        const bool pair = nsweeps - it >= 2;
        for (size_t gi = 0; gi < bt->groups.size(); ++gi) {
            Group& gr = bt->groups[gi];
            if (gr.tier) continue;
            const bool two = gr.pairs;
            if (two && !pair) continue;
            const int runs = (two || !pair) ? 1 : 2;
            for (int r = 0; r < runs; ++r) {
                if ((st = launch_batch_sweep(gr.dtype, gr.stencil, gr.variant, gr.dev,
                                             (int)gr.host.size(), gr.items, phase[gi], two, s)) !=
                    CS_OK)
                    return st;
                phase[gi] ^= 1;
            }
        }
        if (!pair) {
            // the last, odd sweep: the paired groups take it as a single sweep
            for (size_t gi = 0; gi < bt->groups.size(); ++gi) {
                Group& gr = bt->groups[gi];
                if (!gr.pairs) continue;
                if ((st = launch_batch_sweep(gr.dtype, gr.stencil, gr.variant, gr.dev,
                                             (int)gr.host.size(), gr.items, phase[gi], false, s)) !=
                    CS_OK)
                    return st;
                phase[gi] ^= 1;
            }
        }
        it += pair ? 2 : 1;
    }
    for (size_t gi = 0; gi < bt->groups.size(); ++gi) {
        Group& gr = bt->groups[gi];
        if (phase[gi] &&
            (st = launch_batch_copyback(gr.dtype, gr.dev, (int)gr.host.size(), gr.res_items, s)) != CS_OK)
            return st;
    }
    return CS_OK;
}

cs_status cs_batch_sweeps_per_pass(cs_batch bt, int32_t index, int32_t* out)
{
    if (!bt || !out) { set_error("NULL argument"); return CS_EINVAL; }
    if (index < 0 || index >= bt->count) { set_error("patch index out of range"); return CS_EINVAL; }
    *out = bt->per_pass[(size_t)index];
    return CS_OK;
}

cs_status cs_batch_residual(cs_batch bt, double* norms, void* stream)
{
    if (!bt) { set_error("batch is NULL"); return CS_EINVAL; }
    if (bt->count == 0) return CS_OK;
    cs_status st = check_device_range_pub(norms, sizeof(double) * 3 * (size_t)bt->rows,
                                          sizeof(double), "norms");
    if (st != CS_OK) return st;
    for (auto& gr : bt->groups)
        if ((st = launch_batch_residual(gr.dtype, gr.stencil, gr.dev, (int)gr.host.size(),
                                        gr.res_items, bt->partials + gr.partial_base, norms,
                                        (hipStream_t)stream)) != CS_OK)
            return st;
    return CS_OK;
}

}  // extern "C"
