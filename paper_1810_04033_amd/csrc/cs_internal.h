// Internal declarations of the colsten host library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/colsten.h"

namespace cs {

// Geometry passed by value to every kernel.
struct Geo {
    int64_t nx, ny, nz;  // interior points (nz == 1 in 2D)
    int64_t sy, sz;      // element strides (sz == 0 in 2D)
    int parity;
};

// Cost of the expensive stencil evaluation S(k): kmax sin evaluations per
// entry (hetero: linearly 0..kmax-1 over the lexicographic interior index of
// npts points); zero, a, c are the run-time constants of the added terms.
struct StencilCost {
    int kmax;
    int hetero;
    int64_t npts;
    double zero, a, c;
};

// Residual partial sums written by each block of the first reduction stage.
struct Partial {
    double sum_r2;
    double max_r;
    double sum_b2;
};

// Largest number of first-stage residual blocks (fixed, so the reduction
// order does not depend on anything but the grid shape).
constexpr int kMaxResidualBlocks = 2048;

void set_error(const char* fmt, ...);
// Argument checks shared by the create calls (api.hip).
cs_status check_device_range_pub(const void* p, size_t bytes, size_t align, const char* name);
cs_status validate_desc_pub(const cs_grid_desc* d);
int64_t span_of_pub(const cs_grid_desc& d);
cs_status hip_fail(hipError_t e, const char* what);
// Maps the last launch error to CS_EHIP (and records it); CS_OK otherwise.
cs_status check_launch(const char* what);

// ---- launchers (kernels in k_basic.hip / k_fused.hip) --------------------
// dtype 0 = double, 1 = float.  All return CS_OK or CS_EHIP.
cs_status launch_colour_pass(int dtype, int dim, int stencil, const Geo& g, void* u,
                             const void* b, double h2, int colour, hipStream_t s,
                             const StencilCost* cost = nullptr);
cs_status launch_fill_uniform(int dtype, int dim, const Geo& g, void* a, uint64_t seed, hipStream_t s);
cs_status launch_apply(int dtype, int dim, int stencil, const Geo& g, const void* u, void* y,
                       double h2, int cellwise, hipStream_t s);
cs_status launch_lex_sweep(int dtype, int dim, int stencil, const Geo& g, void* u, const void* b,
                           double h2, hipStream_t s);
cs_status launch_jacobi(int dtype, int dim, int stencil, const Geo& g, const void* src,
                        void* dst, const void* b, double h2, double omega, hipStream_t s);
cs_status launch_halo_copy(int dtype, int dim, const Geo& g, const void* src, void* dst,
                           hipStream_t s);
cs_status launch_interior_copy(int dtype, int dim, const Geo& g, const void* src, void* dst,
                               hipStream_t s);
cs_status launch_residual(int dtype, int dim, int stencil, const Geo& g, const void* u,
                          const void* b, void* r, double h2, Partial* partials,
                          double* norms, hipStream_t s);
// One fused Gauss-Seidel sweep src -> dst (3D grids); returns
// CS_EUNSUPPORTED for shapes the fused kernels do not cover.
// src_pairs: src admits two-column loads (pair_layout), used by the 27-point
// sweep where given.
cs_status launch_fused_sweep(int dtype, int dim, int stencil, const Geo& g, const void* src,
                             void* dst, const void* b, double h2, hipStream_t s,
                             bool src_pairs = false);
// Whether an array of the grid's layout at p, with room_before / room_after
// bytes of its allocation before p and after its span, admits the 27-point
// sweep's two-column loads: odd columns aligned to two elements, even strides,
// a padding element after every row, and one element of the allocation before
// p and after the span (the loads of the pairs (-1, 0) and (nx+1, nx+2)).
bool pair_layout(const Geo& g, int dim, const void* p, size_t elem, size_t room_before, size_t room_after);
bool fused_supported(int dtype, int dim, int stencil, const Geo& g);
// Two red-black sweeps (7-point, 3D) in one pass over memory, src -> dst: the
// iterate of two fused sweeps bit for bit.  Available on every 7-point grid
// the fused sweep supports; preferred where the grid is also large enough for
// the double sweep to be the faster choice.
bool fused_two_available(int dtype, int dim, int stencil, const Geo& g);
// Fused sweeps of 2D grids (k_fused2d.hip): sweeps (1 or 2, or 4 for the
// 5-point stencil) whole sweeps per launch, src -> dst.
int fused2d_max_sweeps(int stencil);
// Weighted Jacobi sweeps of 2D grids, sweeps (1, 2, 4 or 8) per launch on an
// LDS-resident tile, src -> dst; the most this grid is run with.
int jacobi2d_max_sweeps(const Geo& g);
cs_status launch_jacobi2d(int dtype, int stencil, int sweeps, const Geo& g, const void* src,
                          void* dst, const void* b, double h2, double omega, hipStream_t s);
cs_status launch_fused2d(int dtype, int stencil, int sweeps, const Geo& g, const void* src,
                         void* dst, const void* b, double h2, hipStream_t s);
bool fused_two_preferred(int dtype, int dim, int stencil, const Geo& g);
cs_status launch_fused_two(int dtype, int dim, int stencil, const Geo& g, const void* src,
                           void* dst, const void* b, double h2, hipStream_t s);
// Second (fixed-order) stage of the residual reduction over `count` partials.
cs_status launch_residual_finish(const Partial* partials, int count, double* norms, hipStream_t s);
// Mixed-precision refinement: FP64 residual with the scaled FP32 copy and
// e32 = 0 (g2 is the FP32 layout), and x += e32 * scale.
cs_status launch_ir_residual(int dim, int stencil, const Geo& g, const void* x, const void* b,
                             double h2, double inv_scale, const Geo& g2, void* r32, void* e32,
                             Partial* partials, double* norms, hipStream_t s);
cs_status launch_ir_residual3(int stencil, const Geo& g, const void* x, const void* b, double h2,
                              double inv_scale, const Geo& g2, void* r32, void* e32,
                              Partial* partials, double* norms, hipStream_t s);
cs_status launch_ir_update(int dim, const Geo& g, void* x, const Geo& g2, const void* e32,
                           double scale, hipStream_t s);
// Persistent colour sweeps with a device-wide barrier between colours
// (k_sync.hip); bar: three zeroed words of device memory owned by the grid.
// The Hyb-depend form (k_sync.hip): tiles wait for their neighbours' previous
// colour phase through per-tile counters in bar[4 ..]; bar[2] counts waits
// that gave up, bar[3] is the abort flag.
void dep_tile_counts(const Geo& g, int dim, int64_t* tnx, int64_t* tny, int64_t* tnz);
cs_status launch_dep_sweeps(int dtype, int dim, int stencil, const Geo& g, void* u, const void* b,
                            double h2, int nsweeps, unsigned* bar, hipStream_t s);
// All sweeps of a small grid in one workgroup, a workgroup barrier per colour
// (k_sync.hip); the iterate of the colour passes.
cs_status launch_block_sweeps(int dtype, int dim, int stencil, const Geo& g, void* u,
                              const void* b, double h2, int nsweeps, hipStream_t s);
cs_status launch_sync_sweeps(int dtype, int dim, int stencil, const Geo& g, void* u,
                             const void* b, double h2, int nsweeps, unsigned* bar, hipStream_t s);
// z-streaming Jacobi and residual for 3D grids (k_stream.hip).
bool stream_supported(const Geo& g);
bool residual3_stream_fits(const Geo& g);
cs_status launch_jacobi3_stream(int dtype, int stencil, const Geo& g, const void* src, void* dst,
                                const void* b, double h2, double omega, hipStream_t s);
// Two Jacobi sweeps in one pass over memory (3D): src -> dst holds the
// iterate of two one-sweep passes bit for bit.
bool jacobi3_two_supported(int stencil, const Geo& g);
cs_status launch_jacobi3_two(int dtype, int stencil, const Geo& g, const void* src, void* dst,
                             const void* b, double h2, double omega, hipStream_t s);
cs_status launch_residual3_stream(int dtype, int stencil, const Geo& g, const void* u,
                                  const void* b, void* r, double h2, Partial* partials,
                                  double* norms, hipStream_t s);

}  // namespace cs

namespace cs {
// A node of the nested-dissection tree (k_nd.hip): the box lo..hi (interior
// coordinates), the cut axes (bit a: axis a cut at m[a]); cut == 0 is a leaf.
struct NdNode {
    int32_t lo[3], hi[3], m[3];
    int32_t cut;
};
}  // namespace cs

namespace cs {
// Multigrid transfers (k_mg.hip): full weighting of the fine residual r into
// the coarse b (and zero into the coarse u), d-linear interpolation of the
// coarse u added to the fine u.
cs_status launch_restrict(int dtype, int dim, const Geo& gf, const void* r, const Geo& gc,
                          void* bc, void* uc, hipStream_t s);
cs_status launch_prolong_add(int dtype, int dim, const Geo& gc, const void* uc, const Geo& gf,
                             void* uf, hipStream_t s);
}  // namespace cs

#include <vector>
namespace cs {
// The dissection tree of a grid, grouped by height (leaves first), and the
// sweeps in that ordering (k_nd.hip).
cs_status nd_tree(const Geo& g, int dim, int64_t leaf, std::vector<NdNode>* nodes,
                  std::vector<int>* stage_off);
cs_status launch_nd_sweeps(int dtype, int dim, int stencil, const Geo& g, void* u, const void* b,
                           double h2, int nsweeps, const NdNode* nodes, const int* stage_off,
                           int nstages, hipStream_t s);
}  // namespace cs

struct cs_grid_s {
    cs_grid_desc d;
    cs::Geo geo;
    void* u;
    const void* b;
    int device;
    size_t elem;          // bytes per element
    int64_t span;         // elements from the first to one past the last halo'd element
    cs::Partial* partials;  // kMaxResidualBlocks entries of device scratch
    int pass_mode;        // cs_pass_mode: sweeps per pass over memory
    unsigned* bar;        // device-wide barrier words of the persistent sweep
    cs::NdNode* nd_nodes; // nested-dissection tree on the device (built on first use)
    int64_t nd_leaf;      // leaf size it was built for (0: none)
    std::vector<int>* nd_stage_off;  // node offsets per height
    bool pair_loads;      // u admits the two-column loads of the 27-point sweep (pair_layout)
};
