/*
 * colsten.h -- C ABI of the coloured stencil-sweep library for MI355X (gfx950).
 *
 * The operations follow Hazelwood & Weinzierl, "Coloured and task-based
 * stencil codes" (arXiv:1810.04033):
 *   - the mesh is a fixed-size d-dimensional Cartesian grid stored as a plain
 *     d-dimensional array with one scalar per cell (Sec. 2);
 *   - a Gauss-Seidel update computes one value per cell from its own and its
 *     neighbours' values through a fixed stencil and writes it in situ (Sec. 2);
 *   - the stencils are the 2d+1-point finite-difference and 3^d-point d-linear
 *     finite-element families (Fig. 1, Sec. 2);
 *   - colouring (red-black for 2d+1 points, 2^d colours otherwise) orders the
 *     sweep into c passes whose updates are independent (Sec. 3);
 *   - a separate output array turns the same sweep into a mat-vec (Sec. 2),
 *     which is the weighted Jacobi sweep and the residual here.
 *
 * Conventions shared by every call
 * --------------------------------
 * Arrays live in device memory owned by the caller; the library never frees
 * them.  Each array carries a one-point halo on every side holding Dirichlet
 * boundary values; x is contiguous.  Element (i, j, k), 0 <= i <= n[0]+1 etc.,
 * sits at offset i + j*stride[1] + k*stride[2] (k = 0 and no z halo in 2D).
 * Interior points are 1 <= i <= n[0], 1 <= j <= n[1], 1 <= k <= n[2].
 *
 * The operator is A = S / h^2 with the dimensionless stencil S:
 *   CS_FD, d = 2:  5-point,  S_0 = 4,   faces -1
 *   CS_FD, d = 3:  7-point,  S_0 = 6,   faces -1
 *   CS_Q1, d = 2:  9-point,  S_0 = 8/3, all neighbours -1/3
 *   CS_Q1, d = 3:  27-point, S_0 = 8/3, faces 0, edges -1/6, corners -1/12
 *                  (assembled trilinear element stiffness)
 *
 * Colours, with parity p in {0, 1} (p = 1 reproduces Algorithm 1's order):
 *   CS_FD: colour = ((i-1) + (j-1) + (k-1) + p) mod 2       (2 colours)
 *   CS_Q1: colour = sum_m ((x_m - 1 + p) mod 2) * 2^m        (2^d colours)
 * A sweep applies the colours 0, 1, ..., c-1 in this order.
 *
 * Streams: every `stream` argument is a hipStream_t passed as void* (NULL is
 * the default stream).  Work is enqueued asynchronously; nothing here
 * synchronises the host except cs_grid_create/cs_batch_create, which may
 * allocate.  Device faults surface at the caller's next synchronisation.
 *
 * Errors: every call returns a cs_status; CS_OK is 0.  On failure nothing has
 * been enqueued (argument errors are detected before any launch) unless the
 * status is CS_EHIP, and cs_last_error() describes the failure.
 */
#ifndef COLSTEN_H
#define COLSTEN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CS_OK = 0,
    CS_EINVAL = 1,        /* invalid argument (null, size, stride, range) */
    CS_ENOMEM = 2,        /* device allocation failed */
    CS_EHIP = 3,          /* a HIP runtime call or kernel launch failed */
    CS_EUNSUPPORTED = 4   /* valid but not supported combination */
} cs_status;

typedef enum { CS_F64 = 0, CS_F32 = 1 } cs_dtype;
typedef enum { CS_FD = 0, CS_Q1 = 1 } cs_stencil;

/* Geometry and method of one grid.  All fields are read at create time. */
typedef struct cs_grid_desc {
    int32_t dim;        /* 2 or 3 */
    int32_t stencil;    /* cs_stencil */
    int32_t dtype;      /* cs_dtype: element type of u and b */
    int32_t parity;     /* colour parity p, 0 or 1 */
    int64_t n[3];       /* interior points along x, y, z; n[2] must be 1 in 2D */
    int64_t stride[3];  /* element strides; stride[0] == 1,
                           stride[1] >= n[0] + 2,
                           stride[2] >= stride[1] * (n[1] + 2) in 3D (ignored in 2D) */
    double h;           /* mesh width, > 0; A = S / h^2 */
} cs_grid_desc;

typedef struct cs_grid_s* cs_grid;

/* Bind a grid to the caller's arrays u (unknowns, updated in place) and b
 * (right-hand side): the fixed-size d-dimensional mesh with one value per cell
 * of Sec. 2, its stencil from Fig. 1 and its colouring of Sec. 3.  Both must be device allocations on the current device
 * covering the whole halo'd extent; the check uses the allocation's address
 * range.  Allocates a small reduction scratch (freed by cs_grid_destroy).
 * Errors: CS_EINVAL on a bad descriptor or pointer, CS_ENOMEM, CS_EHIP. */
cs_status cs_grid_create(const cs_grid_desc* desc, void* u, const void* b, cs_grid* out);

/* Release the handle and its scratch (not u or b).  NULL is a no-op.  The
 * caller must ensure no work using the grid is still pending. */
cs_status cs_grid_destroy(cs_grid g);

/* Number of colours c: 2 for CS_FD, 2^d for CS_Q1 (Sec. 3). */
cs_status cs_num_colours(cs_grid g, int32_t* out);

/* One Gauss-Seidel colour pass (Sec. 3): every interior point q of the given
 * colour is set to (h^2 b_q - sum_{o != 0} S_o u_{q+o}) / S_0, in place.
 * Points of one colour do not couple, so the pass has no ordering freedom.
 * Errors: CS_EINVAL if colour is outside [0, c). */
cs_status cs_colour_pass(cs_grid g, int32_t colour, void* stream);

/* nsweeps full Gauss-Seidel sweeps, each the colours 0..c-1 in order (the
 * in-situ update of Sec. 2 ordered by the colouring of Sec. 3).
 * u_tmp: NULL, or a caller-owned device array with exactly u's layout.  With
 * u_tmp the library runs the sweeps as fused passes over memory, each reading
 * u (or u_tmp) and writing the other array (the same iterate as the colour
 * passes, rounded identically): one or two sweeps per pass on 3D grids, up to
 * four on 2D grids (see cs_grid_set_pass_mode).  The halo of u_tmp is
 * overwritten with u's halo, and the result ends in u.  Without u_tmp, each
 * sweep is c in-place colour passes.  In the automatic pass mode small 3D
 * grids take faster schedules of the same iterate whatever u_tmp is: by
 * default up to 4096 points every sweep runs in one workgroup with a
 * workgroup barrier after each colour (one launch in all), and 7-point grids
 * of up to 1.1 M points run the in-place colour passes (u_tmp unused in both
 * cases); cs_grid_schedule_policy moves these limits.
 * nsweeps == 0 is a no-op.
 * Errors: CS_EINVAL (nsweeps < 0). */
cs_status cs_gs_sweeps(cs_grid g, int32_t nsweeps, void* u_tmp, void* stream);

/* nsweeps weighted Jacobi sweeps (the separate-output-array form of Sec. 2):
 *   u'_q = u_q + omega * (h^2 b_q - sum_o S_o u_{q+o}) / S_0
 * reading only the previous iterate.  u_tmp (required) must have u's layout;
 * its halo is overwritten with u's halo.  The result ends in u.  The sweeps
 * run two per pass over memory on 3D grids and up to eight per launch on 2D
 * grids (the intermediate iterates stay on chip; see cs_grid_set_pass_mode);
 * the iterate is the same, rounded identically.
 * Errors: CS_EINVAL (u_tmp NULL, nsweeps < 0, omega not finite). */
cs_status cs_jacobi_sweeps(cs_grid g, double omega, int32_t nsweeps, void* u_tmp, void* stream);

/* nsweeps Gauss-Seidel sweeps (colours 0..c-1 in order, in place) in one
 * persistent launch with a device-wide barrier after every colour: the
 * Hyb-sync form of the colouring (Sec. 5, Algorithm 1), one parallel region
 * instead of a launch per colour.  The iterate equals cs_gs_sweeps' bit for
 * bit.  Every workgroup of the cooperative launch is resident and runs the
 * same barriers; a barrier wait that polls too long (it never should) is
 * counted, gives up and goes on instead of hanging -- see
 * cs_gs_sync_failures.  Errors: CS_EINVAL (nsweeps < 0), CS_EHIP if the
 * cooperative launch is refused. */
cs_status cs_gs_sweeps_sync(cs_grid g, int32_t nsweeps, void* stream);

/* *out = number of waits of cs_gs_sweeps_sync and cs_gs_sweeps_dep on g that
 * gave up since the grid was created (0 unless something went wrong).
 * Synchronises stream.
 * Errors: CS_EINVAL (bad grid, out NULL), CS_EHIP. */
cs_status cs_gs_sync_failures(cs_grid g, int32_t* out, void* stream);

/* The Hyb-depend form of the colouring (Sec. 5): nsweeps sweeps in one
 * persistent launch without any barrier between colours.  The grid is cut into
 * tiles (32 x 16 x 8 points in 3D, deepened in z towards one tile per resident
 * workgroup, 64 x 32 in 2D), each with a counter of the
 * colour phases it has finished; a tile runs colour phase p (sweep p / c,
 * colour p % c) once its 8 (2D) or 26 (3D) neighbour tiles have finished phase
 * p - 1, so no tile runs more than one phase ahead of a neighbour and the
 * iterate is that of the colour passes, bit for bit.  Workgroups are kept
 * resident (cooperative launch) and take the tiles round robin.  Each wait is
 * bounded: a wait that gives up is counted (read with cs_gs_sync_failures) and
 * ends all other waits, so the call always returns; the result of such a call
 * is not to be used.  Errors: CS_EINVAL (nsweeps < 0, or more than 2^31 colour
 * phases), CS_EHIP (cooperative launch refused). */
cs_status cs_gs_sweeps_dep(cs_grid g, int32_t nsweeps, void* stream);

/* Gauss-Seidel in the nested-dissection ordering of Sec. 3 (a different
 * iterate from the colouring).  The paper leaves the recursion depth and the
 * order inside a separator open; here a box whose every edge is at most `leaf`
 * cells is a leaf swept in z-y-x order, and otherwise every axis longer than
 * `leaf` is cut at the cell lo + extent / 2, the sub-boxes are processed
 * recursively, then the separator (the cells on a cut) in z-y-x order.  Boxes
 * of the tree that are not nested never couple, so all nodes of one height run
 * in one launch (leaves first): one thread per node in 2D, one workgroup per
 * node in 3D stepping through the node's cells by hyperplanes (the same order
 * for every coupled pair).  The first call on a grid
 * with a given leaf builds the tree on the host and uploads it (one device
 * allocation, a synchronous copy); later calls allocate nothing.  Under graph
 * capture the tree must already exist: a call on a capturing stream whose tree
 * is not built returns CS_EINVAL before touching the stream.
 * Errors: CS_EINVAL (nsweeps < 0, leaf < 1, tree not built under capture),
 * CS_EUNSUPPORTED (sizes beyond 2^30), CS_ENOMEM. */
cs_status cs_gs_sweeps_nd(cs_grid g, int32_t nsweeps, int32_t leaf, void* stream);

/* nsweeps lexicographic Gauss-Seidel sweeps: the iterate of the sequential
 * in-place loop in z-y-x order (x innermost), which the task graph of Sec. 3
 * preserves; no colouring, so a different iterate from cs_gs_sweeps.  Run as
 * hyperplane wavefronts, one launch per hyperplane s = i + j + k (2d+1-point
 * stencils) or s = i + 2j + 4k (3^d-point; 2D drops k), in increasing s:
 * about (1 + 1 + 1) n or (1 + 2 + 4) n launches per sweep for an n^3 grid.
 * The grid's parity is ignored.  Errors: CS_EINVAL (nsweeps < 0). */
cs_status cs_gs_sweeps_lex(cs_grid g, int32_t nsweeps, void* stream);

/* nsweeps Gauss-Seidel sweeps (colour passes 0..c-1, one launch each) with
 * the expensive stencil evaluation S(k) of Sec. 2, sized as in Sec. 4: every
 * nonzero stencil entry of every update is recomputed from k evaluations of
 * sin whose contributions are exact zeros, so the iterate equals that of
 * cs_gs_sweeps (without u_tmp) bit for bit while the arithmetic per update
 * grows with k.  hetero == 0: k = kmax at every point; hetero == 1:
 * k = floor(kmax * l / N) over the lexicographic interior index l of the N
 * interior points (the load runs linearly over the mesh).
 * Errors: CS_EINVAL (nsweeps < 0, kmax outside [0, 100000], hetero not 0/1). */
cs_status cs_gs_sweeps_cost(cs_grid g, int32_t nsweeps, int32_t kmax, int32_t hetero,
                            void* stream);

/* Seeded input on the device: the interior of a (layout desc, device array)
 * receives i.i.d. uniform[-1, 1) values from SplitMix64 in counter form,
 * value(seed, l) = mix64(seed + (l + 1) * 0x9E3779B97F4A7C15) at lexicographic
 * interior index l (x fastest), as (v >> 11) * 2^-52 - 1 (exact in FP64,
 * rounded for FP32): the same values as the host-side input generator, so a
 * right-hand side can be made where it is used.  The halo is untouched.
 * Errors: CS_EINVAL for a bad descriptor or pointer. */
cs_status cs_fill_uniform(const cs_grid_desc* desc, void* a, uint64_t seed, void* stream);

/* Operator application y = A u = (S u) / h^2 at the interior points (the
 * separate-output-array mat-vec of Sec. 2).  cellwise == 0: stencil form, the
 * ordered neighbour sum; y's halo is untouched.  cellwise == 1 (d-linear
 * stencils only): the element-wise form, every cell adding its element
 * stiffness times its 2^d vertex values into those vertices, in 2^d cell-colour
 * passes whose cells share no vertex (race-free accumulation into vertices);
 * the same operator up to summation order, and y's halo receives partial sums.
 * y: caller-owned device array with u's layout and dtype, distinct from u and b.
 * Errors: CS_EINVAL (bad y, cellwise not 0/1, cellwise with CS_FD). */
cs_status cs_apply(cs_grid g, void* y, int32_t cellwise, void* stream);

/* Residual r_q = b_q - (S u)_q / h^2 over the interior: the stencil applied
 * into a separate output array (the mat-vec of Sec. 2), subtracted from b.  r: NULL or a device
 * array with u's layout and dtype (halo untouched).  norms: device pointer to
 * 3 doubles receiving ||r||_2, max |r| and ||b||_2 (unweighted sums over
 * interior points), or NULL when only r is wanted (the final reduction is then
 * skipped).  The reduction order is fixed, so repeated calls on the same data
 * give identical bits.  FP32 grids are evaluated in FP64.
 * Errors: CS_EINVAL when r and norms are both NULL or either is bad. */
cs_status cs_residual(cs_grid g, void* r, double* norms, void* stream);

/* The residual of cs_residual for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): no grid handle, no allocation, no host synchronisation.  desc,
 * u, b, r and norms mean what they mean for cs_grid_create and cs_residual
 * (u, b and r device arrays of desc's layout and dtype, r may be NULL, norms
 * may be NULL but not both), validated the same way; the values and their bits
 * equal cs_residual's on a grid of the same descriptor.  The first-stage
 * partial sums live in a fixed array of the library in device memory
 * (2048 x 24 bytes per device, held until the process ends), looked up once per
 * device on the first call made with that device current.  Every grid size the
 * descriptor rules accept fits it: the first reduction stage never uses more
 * than 2048 partials.  Calls that overlap on one device share that array and
 * race; calls on one stream, or otherwise ordered, do not.
 * Errors: as cs_residual, plus CS_EINVAL for a bad descriptor or array,
 * CS_EUNSUPPORTED for a device ordinal of 64 or more, CS_EHIP if the array's
 * address cannot be looked up. */
cs_status cs_residual_noalloc(const cs_grid_desc* desc, const void* u, const void* b, void* r,
                              double* norms, void* stream);

/* ---- Multigrid grid transfers -------------------------------------------
 * A geometric multigrid V-cycle whose smoother is the coloured Gauss-Seidel
 * sweep (the paper names multigrid as the setting its smoothers serve,
 * Sec. 1).  fine and coarse are grids of the same dim, stencil and dtype with
 * fine n = 2 * coarse n + 1 along every axis; fine index i = 2 I lies on
 * coarse index I (vertex-centred), so the coarse halo lies on the fine halo.
 * The coarse grid carries the correction equation A_2h e = R r: its h is
 * expected to be twice the fine h (not checked; the transfers do not use h).
 *
 * cs_restrict: coarse.b <- R r by full weighting at every coarse interior
 *   point, sum over o in {-1,0,1}^d of prod_m w(o_m) r(2I + o), w(0) = 1/2,
 *   w(+-1) = 1/4, in lexicographic (oz, oy, ox) order with one fused
 *   multiply-add per term; coarse.u <- 0 at the same points (halos
 *   untouched).  r: device array with fine u's layout and dtype (e.g. the r
 *   of cs_residual), read at fine interior points only; it must not be
 *   fine.u or one of coarse's arrays.  coarse.b is written although the grid
 *   otherwise only reads b.
 * cs_prolong_add: fine.u <- fine.u + P coarse.u at every fine interior point,
 *   P the d-linear interpolation: the 1, 2, 4 or 8 coarse values around i / 2
 *   (coarse halo included, so the halo of a correction must hold zeros),
 *   weighted 1 or 1/2 per axis, summed in increasing (cz, cy, cx) order with
 *   one fused multiply-add per term, then one addition.
 * Both are deterministic; both ask nothing of the grids' colouring parity.
 * Errors: CS_EINVAL for mismatched grids or sizes, arrays shared between the
 * two grids, or a bad r. */
cs_status cs_restrict(cs_grid fine, const void* r, cs_grid coarse, void* stream);
cs_status cs_prolong_add(cs_grid coarse, cs_grid fine, void* stream);

/* ---- FP32 sweeps inside FP64 iterative refinement ----------------------
 * The paper computes in FP64 only (Sec. 2); these two calls wrap its coloured
 * sweep (Sec. 3) run in FP32 into an FP64 refinement loop.  g64: an FP64 grid whose u holds the iterate x and whose b is the right-hand
 * side.  g32: an FP32 grid of the same dim, stencil, parity, n and h (its own
 * strides) whose u holds the correction e and whose b array receives the
 * scaled residual.  One refinement step is
 *   cs_ir_residual(g64, g32, s)   r = b - A x (FP64); g32.b = fl32(r / s);
 *                                 g32.u = 0 on the interior; norms of r
 *   cs_gs_sweeps(g32, m, ...)     m FP32 Gauss-Seidel sweeps on A e = r / s
 *   cs_ir_update(g64, g32, s)     x <- x + s * e (FP64)
 * scale s must be a positive power of two (then r / s and s * e are exact)
 * and is chosen by the caller, e.g. from the previous step's max |r|.  The
 * residual and the update stay in FP64 on the device.  norms: device pointer
 * to 3 doubles as in cs_residual.  Errors: CS_EINVAL on mismatched grids, a
 * scale that is not a power of two, or a bad norms pointer. */
cs_status cs_ir_residual(cs_grid g64, cs_grid g32, double scale, double* norms, void* stream);
cs_status cs_ir_update(cs_grid g64, cs_grid g32, double scale, void* stream);

/* ---- Batched patches ----------------------------------------------------
 * Many independent 3D patches (the regular patches of block-structured
 * meshes, Sec. 1-2, each swept by the colouring of Sec. 3), each with its own descriptor (n, strides, h, parity),
 * its own u and b, and a work array tmp with u's layout; stencil and dtype
 * may differ between patches.  Patches are grouped by (stencil, dtype, tile
 * variant) and every sweep is one launch per group covering all its patches.
 * All pointers are validated like cs_grid_create's; the descriptor tables are
 * uploaded (synchronously) at create.  The arrays stay owned by the caller
 * and must outlive the batch. */
typedef struct cs_batch_s* cs_batch;

cs_status cs_batch_create(const cs_grid_desc* descs, void* const* u, const void* const* b,
                          void* const* tmp, int32_t count, cs_batch* out);
cs_status cs_batch_destroy(cs_batch bt);

/* A batch whose patches change over time without allocation or host
 * synchronisation (the active set of a request server): cs_batch_reserve
 * allocates, once, device tables for up to `capacity` patches, room for
 * `partials` residual partial sums (a patch needs ceil(n[1] n[2] / 16)) and
 * two pinned host staging buffers; the batch starts empty.  cs_batch_assign
 * replaces its patches (same arguments and checks as cs_batch_create, plus
 * `rows`): the tables are written into a staging buffer and copied to the
 * device asynchronously on `stream`, so the batch must then be used on that
 * stream (or after it).  A staging buffer is reused only once the copy that
 * last read it has run, so an assignment waits only when two earlier ones
 * are still queued.  rows: NULL (patch i reports in norms row i) or one
 * distinct row >= 0 per patch, the row in the norms (and scales) arrays of
 * cs_batch_residual and cs_batch_ir_*, so a patch keeps its row while others
 * come and go.  Errors: CS_EINVAL (capacity or partials exceeded, bad
 * patch, repeated row), CS_ENOMEM (reserve), CS_EHIP. */
cs_status cs_batch_reserve(int32_t capacity, int64_t partials, cs_batch* out);
cs_status cs_batch_assign(cs_batch bt, const cs_grid_desc* descs, void* const* u, const void* const* b,
                          void* const* tmp, const int32_t* rows, int32_t count, void* stream);

/* FP32 sweeps inside FP64 iterative refinement for every patch of an FP32
 * batch at once (the batched form of cs_ir_residual / cs_ir_update).
 * cs_batch_ir_attach pairs each patch of bt (in its assignment order; its u is
 * the correction e, its b receives the scaled residual) with an FP64 patch
 * of the same n and stencil: its iterate x and right-hand side b (descs64,
 * any strides).  Copied asynchronously on stream like cs_batch_assign; a new
 * assignment drops the pairing.
 * cs_batch_ir_residual: for every patch, with row r, s = the smallest power of
 * two >= norms[3 r + 1] (the previous max |r|; put max |b| there before the
 * first step), scales[r] = s, then r = b - A x (FP64), r32 = fl32(r / s),
 * e = 0 on the interior, and norms[3 r .. 3 r + 2] = ||r||_2, max |r|, ||b||_2.
 * cs_batch_ir_update: x <- x + scales[r] * e (FP64) for every patch.
 * One refinement step is update, residual, then m FP32 sweeps of bt
 * (cs_batch_gs_sweeps); e = 0 makes the first update exact.  norms and scales
 * are device arrays of 3 and 1 doubles per row.  Each patch's values are
 * computed from its own data only, as cs_ir_residual and cs_ir_update compute
 * them (norms summed in a different order).
 * Errors: CS_EINVAL (mismatched patches, no pairing, bad arrays). */
cs_status cs_batch_ir_attach(cs_batch bt, const cs_grid_desc* descs64, void* const* x,
                             const void* const* b, void* stream);
cs_status cs_batch_ir_residual(cs_batch bt, double* scales, double* norms, void* stream);
cs_status cs_batch_ir_update(cs_batch bt, const double* scales, void* stream);

/* nsweeps Gauss-Seidel sweeps of every patch (colours in canonical order).
 * Patches small enough to live in one workgroup's LDS (by default up to about
 * 24^3 in FP64 and 32^3 in FP32, see cs_batch_resident_policy) run all nsweeps
 * sweeps in one launch, one workgroup per patch, the patch loaded once,
 * swept colour by colour in LDS with a workgroup barrier after each colour,
 * and written back to u.  Patches of at most 2^17 points whose halo'd
 * cross-section fits at least six (7-point) or seven (27-point) times in LDS
 * (up to about 55 x 55 in FP64), when the batch holds enough of them (see
 * cs_batch_resident_policy), also run all sweeps in one launch, one
 * workgroup per patch:
 * it streams through z with 2 or 3 sweeps per pass, the later sweeps trailing
 * by two planes, in place in u.  Small groups of the remaining patches are
 * swept one colour at a time in place (see cs_batch_colour_policy).  The other
 * patches read their u / tmp alternately,
 * one launch per tile group and pass; the result ends in u (one copy back
 * where a patch's last pass wrote tmp).  Patches of the large 7-point tile
 * class run two red-black sweeps per pass (an odd last sweep alone).  Every
 * schedule gives the same iterate, rounded identically.  The halo of every
 * tmp of a tiled patch is overwritten with u's. */
cs_status cs_batch_gs_sweeps(cs_batch bt, int32_t nsweeps, void* stream);

/* *out = sweeps per pass over memory (1, 2 or 3) of patch index (the caller's
 * order) in cs_batch_gs_sweeps (1 also for the colour passes, one launch per
 * colour), or 0 for a patch swept resident in LDS (all sweeps of a call in
 * one pass).  Errors: CS_EINVAL (NULL, index out of
 * range). */
cs_status cs_batch_sweeps_per_pass(cs_batch bt, int32_t index, int32_t* out);

/* Per-patch residual norms: norms (device, 3 doubles per row) receives, for
 * patch i at 3 * row(i) (row i unless assigned otherwise), ||r||_2, max |r| and
 * ||b||_2 of r = b - A u (FP64 arithmetic).  Each patch's reduction order depends only on its own shape,
 * so its norms do not depend on the rest of the batch. */
cs_status cs_batch_residual(cs_batch bt, double* norms, void* stream);

/* Tile policy for batches created or assigned afterwards (process-wide, per
 * stencil and dtype): a tiled patch with n[0] <= small_max uses the small
 * tile, n[0] <= mid_max the middle one, else the large one (7-point: 16x16,
 * 32x16, 64x16; 27-point: 16x8, 32x16, 64x16).  Default 0, 0 (large tiles
 * only).  Set by the autotuner.  Errors: CS_EINVAL for a bad stencil or
 * dtype, or small_max > mid_max. */
cs_status cs_batch_tile_policy(int32_t stencil, int32_t dtype, int32_t small_max, int32_t mid_max);

/* Colour schedule for batches created afterwards (process-wide, per stencil
 * and dtype): pair_large = 1 (default) runs the sweeps of the large 7-point
 * tile class two per pass over memory, 0 one per pass; the iterate is the same
 * either way.  Set by the autotuner.  Errors: CS_EINVAL for a bad stencil or
 * dtype, or pair_large not 0/1. */
cs_status cs_batch_pass_policy(int32_t stencil, int32_t dtype, int32_t pair_large);

/* Colour-pass schedule for batches created or assigned afterwards
 * (process-wide, per stencil and dtype): a group of tiled patches (one
 * stencil, dtype and tile class) with fewer than max_points interior points in
 * all is swept one colour at a time instead (Sec. 3: one launch per colour,
 * an x-parity pair of colours for the 27-point stencil), in place in u, so
 * that a group too small to give the tile kernels enough work items still
 * spreads over the device.  0 turns it off, -1 restores the default (7-point:
 * 1.25 x 2^20 points in FP64, 1.5 x 2^20 in FP32; 27-point: 2^20 in FP64,
 * 2^22 in FP32).  The iterate is the same either way.  Errors: CS_EINVAL for a bad stencil or dtype, or
 * max_points < -1. */
cs_status cs_batch_colour_policy(int32_t stencil, int32_t dtype, int64_t max_points);

/* Resident schedules for batches created or assigned afterwards
 * (process-wide, per stencil and dtype), a bit mask: bit 0 sweeps every patch
 * that fits one workgroup's LDS and registers resident there; bit 1 streams
 * the patches whose cross-section fits through one workgroup when the batch
 * holds at least one such patch of the stencil and dtype for every compute
 * unit of the device (fewer would leave most of it idle); bit 2 streams them
 * whatever their number.  Resident and streamed patches run all sweeps of a
 * call in one launch; the others go to the tile kernels.  Default 3; the
 * iterate is the same under every mask.  Set by the autotuner.  Errors:
 * CS_EINVAL for a bad stencil or dtype, or a mask outside [0, 7]. */
cs_status cs_batch_resident_policy(int32_t stencil, int32_t dtype, int32_t enable);

/* ---- Captured sweep sequences (HIP graphs) -------------------------------
 * A fixed number of sweeps recorded once into a HIP graph and replayed with
 * one launch call, for callers that repeat the same sweeps many times on small
 * grids, batches or the hyperplane wavefronts, where per-kernel launch cost
 * dominates.  The graph captures the grid's (or batch's) arrays, which must
 * stay allocated until cs_graph_destroy; each launch continues from the
 * current contents of u.  Capture uses a private stream of the library and
 * records kernel nodes only. */
typedef struct cs_graph_s* cs_graph;

/* Record nsweeps sweeps of g: cs_gs_sweeps(g, nsweeps, u_tmp) if
 * lexicographic == 0, cs_gs_sweeps_lex(g, nsweeps) if 1 (u_tmp must then be
 * NULL).  Errors: CS_EINVAL (nsweeps < 1, bad flag), the errors of the
 * recorded call, CS_EHIP if capture or instantiation fails. */
cs_status cs_graph_gs(cs_grid g, int32_t nsweeps, void* u_tmp, int32_t lexicographic, cs_graph* out);

/* Record cs_batch_gs_sweeps(bt, nsweeps). */
cs_status cs_graph_batch_gs(cs_batch bt, int32_t nsweeps, cs_graph* out);

/* Record any sequence of library calls (e.g. a multigrid V-cycle):
 * cs_graph_begin returns a private stream of the library that is capturing
 * (thread-local mode); the caller enqueues library calls on it from the same
 * thread, then cs_graph_end stops the capture, releases the stream and
 * instantiates the graph.  Only the library's own calls belong in between (they
 * record kernel nodes only); their arrays must stay allocated until
 * cs_graph_destroy.  A call that fails in between still needs cs_graph_end,
 * which then reports CS_EHIP if the capture was invalidated.
 * Errors: CS_EINVAL (NULL arguments, a stream that is not capturing), CS_EHIP. */
cs_status cs_graph_begin(void** capture_stream);
cs_status cs_graph_end(void* capture_stream, cs_graph* out);

/* Enqueue one replay on stream (same device as the capture). */
cs_status cs_graph_launch(cs_graph gr, void* stream);

/* Release the graph.  NULL is a no-op; pending replays must have finished. */
cs_status cs_graph_destroy(cs_graph gr);

/* *out = 1 if cs_gs_sweeps with a work array runs this grid's sweeps as fused
 * passes over memory, 0 if it falls back to one launch per colour. */
cs_status cs_gs_fused(cs_grid g, int32_t* out);

/* Sweeps per pass over memory.  Two sweeps in one pass keep the intermediate
 * iterate on chip, so they move the bytes of one sweep; the iterate is the
 * same in every mode, rounded identically (not from the paper, which times
 * single sweeps: a schedule of the same computation).
 *   CS_PASS_AUTO (default): two per pass for 3D Jacobi sweeps and, where the
 *     grid is large enough for it to be faster, for fused 3D red-black sweeps;
 *     one otherwise.  Where a red-black count would take an odd number of
 *     passes, one double pass runs as two single ones, so that the iterate
 *     ends in u without a copy (e.g. 2 sweeps: two single passes).  Fused 2D
 *     sweeps run up to 4 (red-black) or 2 (four colours) per pass.
 *   CS_PASS_ONE: one sweep per pass.
 *   CS_PASS_TWO: as CS_PASS_AUTO, but two 3D sweeps per pass wherever a kernel
 *     for it exists (3D Jacobi, fused 3D red-black and 8-colour), whatever the
 *     grid size.
 * A remainder of sweeps runs in smaller passes.  The fused 3D 8-colour sweeps
 * run one per pass unless CS_PASS_TWO asks for two (their double pass, the
 * second sweep trailing the first by two planes, gives the same iterate but
 * was measured slower on MI355X). */
typedef enum { CS_PASS_AUTO = 0, CS_PASS_ONE = 1, CS_PASS_TWO = 2 } cs_pass_mode;

/* Set the grid's pass mode (a cs_pass_mode).  Errors: CS_EINVAL (bad grid or
 * mode). */
cs_status cs_grid_set_pass_mode(cs_grid g, int32_t mode);

/* Automatic schedule of cs_gs_sweeps on 3D grids in CS_PASS_AUTO
 * (process-wide, per stencil and dtype; the colour order of Sec. 3 in every
 * schedule, so the iterate is the same in all of them): grids of at most
 * block_max interior points run every sweep in one workgroup, grids of at
 * most colour_max points one launch per colour (in place, u_tmp unused),
 * larger ones fused passes with u_tmp, two sweeps per pass from two_min
 * points on where the double sweep is built.  A negative value restores that
 * field's default: block_max 4096; colour_max 1.1 M points (7-point) or 0
 * (27-point); two_min: 7-point where the grid fills the device, 27-point
 * never.  Set by the autotuner.  Errors: CS_EINVAL (bad stencil or dtype). */
cs_status cs_grid_schedule_policy(int32_t stencil, int32_t dtype, int64_t block_max, int64_t colour_max,
                                  int64_t two_min);

/* *out = sweeps per pass (1, 2, 4 or 8; more than 2 only on 2D grids) that cs_gs_sweeps with a work array
 * (jacobi == 0) or cs_jacobi_sweeps (jacobi == 1) uses on this grid under its
 * pass mode.  Errors: CS_EINVAL (bad grid, out NULL, jacobi not 0/1). */
cs_status cs_sweeps_per_pass(cs_grid g, int32_t jacobi, int32_t* out);

/* Description of the last failure on the calling thread ("" if none). */
const char* cs_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* COLSTEN_H */
