// C ABI of the batched patches: validation, grouping, device tables and the
// per-sweep launches.
#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "cs_batch.h"

using namespace cs;

namespace {

struct Group {
    int dtype = 0, stencil = 0, variant = 0;
    int tier = 0;        // LDS-resident tier (1, 2), or 0 for the tile kernels
    bool pairs = false;  // two sweeps per launch
    std::vector<BatchPatch> host;
    BatchPatch* dev = nullptr;
    int64_t items = 0, res_items = 0, partial_base = 0;
};

// [stencil][dtype]
int g_small_max[2][2] = {{16, 16}, {16, 16}};
int g_mid_max[2][2] = {{40, 40}, {40, 40}};
int g_pair_large[2][2] = {{1, 1}, {1, 1}};  // pair the sweeps of the large tile class
int g_resident[2][2] = {{1, 1}, {1, 1}};    // sweep patches that fit in LDS there

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

}  // namespace

struct cs_batch_s {
    int count = 0;
    int device = 0;
    std::vector<Group> groups;
    std::vector<int> per_pass;  // sweeps per launch of each patch (caller's order)
    Partial* partials = nullptr;
};

static void free_batch(cs_batch_s* bt)
{
    if (!bt) return;
    for (auto& gr : bt->groups)
        if (gr.dev) (void)hipFree(gr.dev);
    if (bt->partials) (void)hipFree(bt->partials);
    delete bt;
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

cs_status cs_batch_resident_policy(int32_t stencil, int32_t dtype, int32_t enable)
{
    if ((stencil != CS_FD && stencil != CS_Q1) || (dtype != CS_F64 && dtype != CS_F32) ||
        (enable != 0 && enable != 1)) {
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
    cs_batch_s* bt = new (std::nothrow) cs_batch_s();
    if (!bt) { set_error("out of host memory"); return CS_ENOMEM; }
    bt->count = count;
    if (hipGetDevice(&bt->device) != hipSuccess) { free_batch(bt); return hip_fail(hipGetLastError(), "hipGetDevice"); }
    std::vector<BatchPatch> all;
    std::vector<int> gid;
    for (int32_t i = 0; i < count; ++i) {
        const cs_grid_desc& d = descs[i];
        cs_status st = validate_desc_pub(&d);
        if (st != CS_OK) { free_batch(bt); return st; }
        if (d.dim != 3) { set_error("patch %d: batches hold 3D patches", i); free_batch(bt); return CS_EUNSUPPORTED; }
        if ((d.n[1] + 2) * d.stride[1] >= ((int64_t)1 << 31)) {
            set_error("patch %d: plane too large for 32-bit offsets", i);
            free_batch(bt);
            return CS_EUNSUPPORTED;
        }
        const size_t elem = d.dtype == CS_F64 ? 8 : 4;
        const size_t bytes = (size_t)span_of3(d) * elem;
        if ((st = check_device_range_pub(u[i], bytes, elem, "patch u")) != CS_OK ||
            (st = check_device_range_pub(b[i], bytes, elem, "patch b")) != CS_OK ||
            (st = check_device_range_pub(tmp[i], bytes, elem, "patch tmp")) != CS_OK) {
            free_batch(bt);
            return st;
        }
        if (u[i] == tmp[i] || u[i] == b[i] || tmp[i] == b[i]) {
            set_error("patch %d: u, b and tmp must be separate arrays", i);
            free_batch(bt);
            return CS_EINVAL;
        }
        BatchPatch p{};
        p.g.nx = d.n[0];
        p.g.ny = d.n[1];
        p.g.nz = d.n[2];
        p.g.sy = d.stride[1];
        p.g.sz = d.stride[2];
        p.g.parity = d.parity;
        p.u = u[i];
        p.tmp = tmp[i];
        p.b = b[i];
        p.hh = d.h * d.h;
        p.h2 = d.dtype == CS_F32 ? (double)(float)p.hh : p.hh;
        p.index = i;
        const int tier = g_resident[d.stencil][d.dtype] ? batch_resident_tier(d.dtype, d.stencil, p.g) : 0;
        const int variant = tier ? 0 : pick_variant(d.stencil, d.dtype, d.n[0]);
        const bool pairs = !tier && batch_variant_pairs(d.stencil, variant) && g_pair_large[d.stencil][d.dtype];
        int tx = 0, ty = 0;
        batch_variant_tile(d.stencil, variant, &tx, &ty);
        p.tiles_x = (int)((d.n[0] + tx - 1) / tx);
        p.tiles_y = (int)((d.n[1] + ty - 1) / ty);
        p.chunks = 1;  // set below, once the batch's total tile count is known
        p.res_items = (int)batch_residual_items(p.g);
        // group key
        int k = -1;
        for (size_t j = 0; j < bt->groups.size(); ++j)
            if (bt->groups[j].dtype == d.dtype && bt->groups[j].stencil == d.stencil &&
                bt->groups[j].variant == variant && bt->groups[j].pairs == pairs &&
                bt->groups[j].tier == tier)
                k = (int)j;
        if (k < 0) {
            Group gr;
            gr.dtype = d.dtype;
            gr.stencil = d.stencil;
            gr.variant = variant;
            gr.tier = tier;
            gr.pairs = pairs;
            bt->groups.push_back(gr);
            k = (int)bt->groups.size() - 1;
        }
        bt->groups[k].host.push_back(p);
        bt->per_pass.push_back(tier ? 0 : (pairs ? 2 : 1));
    }
    // z chunks: enough work items to fill the GPU (about 2048) when the batch
    // holds few patches, never chunks thinner than 8 planes (16 for the tile
    // class that also runs double sweeps).  The split does not change any
    // value: every point is computed the same way in any tile.
    int64_t total_tiles = 0;
    for (auto& gr : bt->groups)
        if (!gr.tier)
            for (auto& p : gr.host) total_tiles += (int64_t)p.tiles_x * p.tiles_y;
    const int64_t want = total_tiles > 0 ? (2048 + total_tiles - 1) / total_tiles : 1;
    for (auto& gr : bt->groups) {
        const int depth = gr.pairs ? 16 : 8;
        for (auto& p : gr.host)
            p.chunks = (int)std::max<int64_t>(1, std::min<int64_t>(want, p.g.nz / depth));
    }
    int64_t partial_total = 0;
    for (auto& gr : bt->groups) {
        std::stable_sort(gr.host.begin(), gr.host.end(), [](const BatchPatch& a, const BatchPatch& c) {
            return a.g.nx * a.g.ny * a.g.nz > c.g.nx * c.g.ny * c.g.nz;
        });
        int64_t it = 0, rit = 0;
        for (auto& p : gr.host) {
            p.item_begin = it;
            it += gr.tier ? 1 : (int64_t)p.tiles_x * p.tiles_y * p.chunks;
            p.res_begin = rit;
            rit += p.res_items;
        }
        if (it > 0x7fffffff || rit > 0x7fffffff) { set_error("batch too large"); free_batch(bt); return CS_EUNSUPPORTED; }
        gr.items = it;
        gr.res_items = rit;
        gr.partial_base = partial_total;
        partial_total += rit;
        hipError_t e = hipMalloc((void**)&gr.dev, sizeof(BatchPatch) * gr.host.size());
        if (e != hipSuccess) { (void)hipGetLastError(); set_error("hipMalloc of the patch table failed"); free_batch(bt); return CS_ENOMEM; }
        e = hipMemcpy(gr.dev, gr.host.data(), sizeof(BatchPatch) * gr.host.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) { cs_status s2 = hip_fail(e, "patch table upload"); free_batch(bt); return s2; }
    }
    hipError_t e = hipMalloc((void**)&bt->partials, sizeof(Partial) * (size_t)partial_total);
    if (e != hipSuccess) { (void)hipGetLastError(); set_error("hipMalloc of the batch partials failed"); free_batch(bt); return CS_ENOMEM; }
    *out = bt;
    return CS_OK;
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
    // LDS-resident groups: every sweep in one launch, in place in u
    for (auto& gr : bt->groups)
        if (gr.tier &&
            (st = launch_batch_resident(gr.dtype, gr.stencil, gr.tier, gr.dev, (int)gr.host.size(),
                                        nsweeps, s)) != CS_OK)
            return st;
    for (auto& gr : bt->groups)
        if (!gr.tier && (st = launch_batch_halo(gr.dtype, gr.dev, (int)gr.host.size(), s)) != CS_OK)
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
    cs_status st = check_device_range_pub(norms, sizeof(double) * 3 * (size_t)bt->count,
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
