// Internal declarations of the batched-patch kernels (not part of the ABI).
#pragma once

#include "cs_internal.h"

namespace cs {

// Array pointers in the device tables are typed as global memory: a pointer
// loaded from memory is otherwise generic, and the kernels would access the
// arrays with flat instructions, which also count against the LDS wait counter
// (every LDS wait would then wait for the prefetched loads as well).
#define CS_GLOBAL __attribute__((address_space(1)))

// One patch of a batch group, as stored in the group's device table.
struct BatchPatch {
    Geo g;
    CS_GLOBAL void* u;        // iterate (the result ends here)
    CS_GLOBAL void* tmp;      // work array with u's layout
    const CS_GLOBAL void* b;  // right-hand side
    double h2;        // h^2 as the sweeps use it (rounded to FP32 for FP32 patches)
    double hh;        // h*h in FP64 (residual)
    int tiles_x, tiles_y, chunks;
    int index;        // row of the patch in the norms (the caller's position by default)
    int stencil, dtype;
    int64_t item_begin;  // first work item of this patch in the sweep launch
    int64_t res_begin;   // first row-block item in the residual / copy launches
    int res_items;
    int64_t halo_begin;  // first plane item in the halo copy (nz + 2 items)
};

// One patch of the refinement pairing of an FP32 batch: the FP64 iterate x
// and right-hand side b, and the FP32 correction e and scaled residual r32
// (the FP32 patch's u and b), in the caller's order.
struct IrPatch {
    Geo g;            // x and b
    Geo g2;           // e and r32
    CS_GLOBAL double* x;
    const CS_GLOBAL double* b;
    CS_GLOBAL float* e;
    CS_GLOBAL float* r32;
    double hh;        // h*h (FP64)
    int stencil;
    int row;          // row in the norms and scales
    int64_t res_begin;
    int res_items;
};

int64_t batch_residual_items(const Geo& g);
void batch_variant_tile(int stencil, int variant, int* tx, int* ty);
// Whether a tile variant can also run two sweeps per launch (the large
// 7-point class: 64 x 16 tiles, the same work items for the single and the
// double sweep); its items are then planned at least 16 planes deep.
bool batch_variant_pairs(int stencil, int variant);
cs_status launch_batch_sweep(int dtype, int stencil, int variant, const BatchPatch* tab, int count,
                             int64_t items, int phase, bool two, hipStream_t s);
// Resident tier of a patch: 1 (small) or 2 (large) when the whole patch fits
// one workgroup's LDS and registers, else 0.
int batch_resident_tier(int dtype, int stencil, const Geo& g);
// All nsweeps sweeps of every patch of a resident group in one launch, one
// workgroup per patch, in place in u.
cs_status launch_batch_resident(int dtype, int stencil, int tier, const BatchPatch* tab, int count,
                                int nsweeps, hipStream_t s);
// Refinement steps of every patch of an IR table: r = b - A x in FP64, with
// the scale s = the smallest power of two >= the row's previous max |r|
// (norms[3 row + 1] on entry) written to scales[row], r32 = fl32(r / s),
// e = 0, and the row's norms; and x += scales[row] * e.
cs_status launch_batch_ir_residual(const IrPatch* tab, int count, int64_t items, Partial* partials,
                                   double* scales, double* norms, hipStream_t s);
cs_status launch_batch_ir_update(const IrPatch* tab, int count, int64_t items, const double* scales,
                                 hipStream_t s);
// Whether a patch is swept by the plane-streaming tier (its whole halo'd
// cross-section fits at least 2 x 2 + 1 + NPL times in LDS), and its launch:
// all nsweeps sweeps, one workgroup per patch, in place in u.
bool batch_planes_fits(int dtype, int stencil, const Geo& g);
int batch_planes_sweeps(int dtype, int stencil, const Geo& g);  // sweeps per pass there
// The small form (two workgroups per compute unit) for patches it fits with
// the same sweeps per pass.
bool batch_planes_small(int dtype, int stencil, const Geo& g);
cs_status launch_batch_planes(int dtype, int stencil, const BatchPatch* tab, int count, int nsweeps,
                              hipStream_t s, bool small);
// Colour-pass tier: work items of a patch, and nsweeps sweeps of a group, one
// launch per colour phase, in place in u.
int64_t batch_colour_items(int stencil, const Geo& g);
cs_status launch_batch_colour(int dtype, int stencil, const BatchPatch* tab, int count, int64_t items,
                              int nsweeps, hipStream_t s);
cs_status launch_batch_halo(int dtype, const BatchPatch* tab, int count, int64_t halo_items, hipStream_t s);
cs_status launch_batch_copyback(int dtype, const BatchPatch* tab, int count, int64_t res_items,
                                hipStream_t s);
cs_status launch_batch_residual(int dtype, int stencil, const BatchPatch* tab, int count,
                                int64_t res_items, Partial* partials, double* norms, hipStream_t s);

}  // namespace cs
