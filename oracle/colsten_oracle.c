/*
 * colsten oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, sequential, deliberately slow CPU implementation of the coloured
 * stencil sweeps of Hazelwood & Weinzierl, "Coloured and task-based stencil
 * codes" (arXiv:1810.04033).  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  The GPU library never links,
 * includes or calls anything here, and this file includes nothing of the GPU
 * library.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -shared -fPIC
 * (no implicit contraction: every operation below, including each explicit
 *  fma() call, is one IEEE-754 round-to-nearest-even operation in the order
 *  written).
 *
 * The colour passes and the Jacobi sweeps carry an OpenMP `parallel for` over
 * the rows (k, j): the paper's BSP colouring, one parallel loop per colour
 * with its implicit barrier (Sec. 3).  Without -fopenmp the pragmas are
 * ignored and the loops run in the order written; with it the result is the
 * same bit for bit, because the points of one colour (and all points of a
 * Jacobi sweep) are updated independently.  The sums of the residual keep
 * their fixed sequential order.
 *
 * Data (paper Sec. 2, "The studied stencil codes"): a d-dimensional Cartesian
 * mesh of fixed size stored as a plain d-dimensional array holding one scalar
 * per cell.  Here every array carries a one-point halo on each side that holds
 * Dirichlet boundary values, x is the contiguous axis, and the element strides
 * (1, sy, sz) may include row/plane padding.  Interior indices run over
 * i in [1,nx], j in [1,ny], k in [1,nz]; in 2D nz == 1 and no z offsets exist.
 *
 * Stencils (paper Fig. 1 and Sec. 2): the 2d+1-point finite-difference family
 * and the 3^d-point d-linear finite-element family.  The operator is
 * A = S / h^2 with S the dimensionless stencil.  Weights S_o by offset o:
 *   FD:       S_0 = 2d, face neighbours -1 (Fig. 1, middle, for d = 2).
 *   Q1, d=2:  S_0 = 8/3, all eight neighbours -1/3 (Fig. 1, right).
 *   Q1, d=3:  S_0 = 8/3, faces 0, edges -1/6, corners -1/12.  The paper does
 *             not print the 27-point entries; these are the assembled
 *             trilinear element stiffness (see og_q1_kref below and the
 *             Gauss-quadrature pin in the tests).
 *
 * Colouring (paper Sec. 3, "Colouring"): red-black for the 2d+1-point
 * stencils, 2^d colours otherwise.  With parity offset p:
 *   FD: colour = ((i-1)+(j-1)+(k-1)+p) mod 2
 *   Q1: colour = sum_m ((x_m-1+p) mod 2) * 2^m     (x_0 = i, x_1 = j, x_2 = k)
 * p = 0 puts the first interior point into colour 0 (the greedy construction
 * in the prose of Sec. 3); p = 1 reproduces the index formula of Algorithm 1,
 * whose pass c = 0 starts at x = 2 on row y = 1.
 *
 * Gauss-Seidel colour pass (Sec. 2: one value per cell from its own and its
 * neighbours' values, written in situ; Sec. 3: one pass per colour): for every
 * interior point q of colour c, z-y-x order with x innermost,
 *     u_q <- (h^2 b_q - sum_{o != 0} S_o u_{q+o}) / S_0
 * where the neighbour sum runs over offsets in lexicographic (oz, oy, ox)
 * order, skips zero weights, and accumulates each term with one fused
 * multiply-add (acc <- fma(S_o, u_{q+o}, acc), one rounding per term; the
 * paper leaves the rounding open).  The quotient by S_0 is the exact quotient
 * rounded once: for the d-linear stencils S_0 = 8/3 has the binary inverse
 * 3/8, so x / S_0 is formed as x * 0.375 (a division by the rounded 8/3 would
 * round twice); the FD centre 2d is exact and divides directly.  A sweep is
 * the colour passes 0..c-1 in order.
 *
 * Separate-output update (Sec. 2: a separate output array as in a mat-vec):
 * weighted Jacobi  u'_q = u_q + w (h^2 b_q - sum_o S_o u_{q+o}) / S_0  (the
 * final multiply-add fused as well) and the residual
 * r_q = b_q - (sum_o S_o u_{q+o}) / h^2, both reading only the old u.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* Stencil weights and colours                                          */
/* ------------------------------------------------------------------ */

/* S_o for offset (ox, oy, oz); stencil 0 = FD (2d+1 points), 1 = Q1 (3^d). */
double og_weight(int stencil, int dim, int ox, int oy, int oz)
{
    int nnz = (ox != 0) + (oy != 0) + (oz != 0);
    if (dim == 2 && oz != 0) return 0.0;
    if (stencil == 0) {
        if (nnz == 0) return 2.0 * dim;
        if (nnz == 1) return -1.0;
        return 0.0;
    }
    if (dim == 2) {
        if (nnz == 0) return 8.0 / 3.0;
        return -1.0 / 3.0;
    }
    if (nnz == 0) return 8.0 / 3.0;
    if (nnz == 1) return 0.0;
    if (nnz == 2) return -1.0 / 6.0;
    return -1.0 / 12.0;
}

/* The same weights rounded once to binary32 (for the FP32 sweeps). */
static float og_weight_f32(int stencil, int dim, int ox, int oy, int oz)
{
    int nnz = (ox != 0) + (oy != 0) + (oz != 0);
    if (dim == 2 && oz != 0) return 0.0f;
    if (stencil == 0) {
        if (nnz == 0) return 2.0f * (float)dim;
        if (nnz == 1) return -1.0f;
        return 0.0f;
    }
    if (dim == 2) {
        if (nnz == 0) return 8.0f / 3.0f;
        return -1.0f / 3.0f;
    }
    if (nnz == 0) return 8.0f / 3.0f;
    if (nnz == 1) return 0.0f;
    if (nnz == 2) return -1.0f / 6.0f;
    return -1.0f / 12.0f;
}

int og_num_colours(int stencil, int dim)
{
    return stencil == 0 ? 2 : (1 << dim);
}

/* Colour of interior point (i, j, k), 1-based; k == 1 in 2D. */
int og_colour(int stencil, int dim, int parity, int64_t i, int64_t j, int64_t k)
{
    if (stencil == 0) {
        int64_t s = (i - 1) + (j - 1) + (dim == 3 ? (k - 1) : 0) + parity;
        return (int)(s & 1);
    }
    int c = (int)((i - 1 + parity) & 1);
    c |= (int)((j - 1 + parity) & 1) << 1;
    if (dim == 3) c |= (int)((k - 1 + parity) & 1) << 2;
    return c;
}

/* Static colour validity: no nonzero off-centre weight may couple two points
 * of the same colour (the race-freedom colouring provides a priori, Sec. 3).
 * Checks every interior point against every offset on an n^d box; returns 1
 * when valid.  colour_rule 0 = the stencil's own rule, 1 = force red-black. */
int og_colouring_valid(int stencil, int dim, int colour_rule, int64_t n)
{
    int zr = dim == 3 ? 1 : 0;
    for (int64_t k = 1; k <= (dim == 3 ? n : 1); ++k)
        for (int64_t j = 1; j <= n; ++j)
            for (int64_t i = 1; i <= n; ++i)
                for (int oz = -zr; oz <= zr; ++oz)
                    for (int oy = -1; oy <= 1; ++oy)
                        for (int ox = -1; ox <= 1; ++ox) {
                            if (ox == 0 && oy == 0 && oz == 0) continue;
                            if (og_weight(stencil, dim, ox, oy, oz) == 0.0) continue;
                            int64_t i2 = i + ox, j2 = j + oy, k2 = k + oz;
                            if (i2 < 1 || i2 > n || j2 < 1 || j2 > n) continue;
                            if (dim == 3 && (k2 < 1 || k2 > n)) continue;
                            int rule = colour_rule == 1 ? 0 : stencil;
                            int c1 = og_colour(rule, dim, 0, i, j, k);
                            int c2 = og_colour(rule, dim, 0, i2, j2, k2);
                            if (c1 == c2) return 0;
                        }
    return 1;
}

/* ------------------------------------------------------------------ */
/* One point update, FP64 and FP32                                      */
/* ------------------------------------------------------------------ */

typedef struct {
    int dim, stencil, parity;
    int64_t nx, ny, nz, sy, sz;
    double h;
} og_grid;

static og_grid og_make(int dim, int stencil, int parity, int64_t nx, int64_t ny,
                       int64_t nz, int64_t sy, int64_t sz, double h)
{
    og_grid g;
    g.dim = dim; g.stencil = stencil; g.parity = parity;
    g.nx = nx; g.ny = ny; g.nz = dim == 3 ? nz : 1;
    g.sy = sy; g.sz = dim == 3 ? sz : 0;
    g.h = h;
    return g;
}

static int64_t og_index(const og_grid* g, int64_t i, int64_t j, int64_t k)
{
    return (g->dim == 3 ? k * g->sz : 0) + j * g->sy + i;
}

/* sum_{o != 0} S_o u_{q+o}, lexicographic (oz, oy, ox), zero weights skipped */
static double og_offsum(const og_grid* g, const double* u, int64_t q)
{
    int zr = g->dim == 3 ? 1 : 0;
    double acc = 0.0;
    for (int oz = -zr; oz <= zr; ++oz)
        for (int oy = -1; oy <= 1; ++oy)
            for (int ox = -1; ox <= 1; ++ox) {
                if (ox == 0 && oy == 0 && oz == 0) continue;
                double w = og_weight(g->stencil, g->dim, ox, oy, oz);
                if (w == 0.0) continue;
                acc = fma(w, u[q + oz * g->sz + oy * g->sy + ox], acc);
            }
    return acc;
}

/* sum over all o (centre included, at its lexicographic place) */
static double og_fullsum(const og_grid* g, const double* u, int64_t q)
{
    int zr = g->dim == 3 ? 1 : 0;
    double acc = 0.0;
    for (int oz = -zr; oz <= zr; ++oz)
        for (int oy = -1; oy <= 1; ++oy)
            for (int ox = -1; ox <= 1; ++ox) {
                double w = og_weight(g->stencil, g->dim, ox, oy, oz);
                if (w == 0.0) continue;
                acc = fma(w, u[q + oz * g->sz + oy * g->sy + ox], acc);
            }
    return acc;
}

static float og_offsum_f32(const og_grid* g, const float* u, int64_t q)
{
    int zr = g->dim == 3 ? 1 : 0;
    float acc = 0.0f;
    for (int oz = -zr; oz <= zr; ++oz)
        for (int oy = -1; oy <= 1; ++oy)
            for (int ox = -1; ox <= 1; ++ox) {
                if (ox == 0 && oy == 0 && oz == 0) continue;
                float w = og_weight_f32(g->stencil, g->dim, ox, oy, oz);
                if (w == 0.0f) continue;
                acc = fmaf(w, u[q + oz * g->sz + oy * g->sy + ox], acc);
            }
    return acc;
}

static float og_fullsum_f32(const og_grid* g, const float* u, int64_t q)
{
    int zr = g->dim == 3 ? 1 : 0;
    float acc = 0.0f;
    for (int oz = -zr; oz <= zr; ++oz)
        for (int oy = -1; oy <= 1; ++oy)
            for (int ox = -1; ox <= 1; ++ox) {
                float w = og_weight_f32(g->stencil, g->dim, ox, oy, oz);
                if (w == 0.0f) continue;
                acc = fmaf(w, u[q + oz * g->sz + oy * g->sy + ox], acc);
            }
    return acc;
}

/* x / S_0, the exact quotient rounded once: x * (3/8) for the d-linear
 * stencils (S_0 = 8/3), x / (2d) for the FD stencils. */
static double og_over_centre(int stencil, int dim, double x)
{
    if (stencil == 1) return x * 0.375;
    return x / (2.0 * dim);
}

static float og_over_centre_f32(int stencil, int dim, float x)
{
    if (stencil == 1) return x * 0.375f;
    return x / (float)(2 * dim);
}

/* Gauss-Seidel point update, in situ. */
static void og_update(const og_grid* g, double* u, const double* b, int64_t q)
{
    double h2 = g->h * g->h;
    double rhs = h2 * b[q];
    double acc = og_offsum(g, u, q);
    u[q] = og_over_centre(g->stencil, g->dim, rhs - acc);
}

static void og_update_f32(const og_grid* g, float* u, const float* b, int64_t q)
{
    float h2 = (float)(g->h * g->h);
    float rhs = h2 * b[q];
    float acc = og_offsum_f32(g, u, q);
    u[q] = og_over_centre_f32(g->stencil, g->dim, rhs - acc);
}

/* ------------------------------------------------------------------ */
/* Gauss-Seidel colour passes and sweeps                                */
/* ------------------------------------------------------------------ */

/* One colour pass: every interior point of colour c, z, y, x order. */
void og_colour_pass_f64(int dim, int stencil, int parity, int64_t nx, int64_t ny,
                        int64_t nz, int64_t sy, int64_t sz, double h,
                        double* u, const double* b, int colour)
{
    og_grid g = og_make(dim, stencil, parity, nx, ny, nz, sy, sz, h);
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t k = 1; k <= g.nz; ++k)
        for (int64_t j = 1; j <= g.ny; ++j)
            for (int64_t i = 1; i <= g.nx; ++i)
                if (og_colour(stencil, dim, parity, i, j, k) == colour)
                    og_update(&g, u, b, og_index(&g, i, j, k));
}

void og_colour_pass_f32(int dim, int stencil, int parity, int64_t nx, int64_t ny,
                        int64_t nz, int64_t sy, int64_t sz, double h,
                        float* u, const float* b, int colour)
{
    og_grid g = og_make(dim, stencil, parity, nx, ny, nz, sy, sz, h);
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t k = 1; k <= g.nz; ++k)
        for (int64_t j = 1; j <= g.ny; ++j)
            for (int64_t i = 1; i <= g.nx; ++i)
                if (og_colour(stencil, dim, parity, i, j, k) == colour)
                    og_update_f32(&g, u, b, og_index(&g, i, j, k));
}

/* The same colour pass, visiting the listed flat indices in the given order.
 * Used to check that the order inside one colour does not matter (Sec. 3:
 * the updates within a pass are embarrassingly parallel). */
void og_update_points_f64(int dim, int stencil, int parity, int64_t nx, int64_t ny,
                          int64_t nz, int64_t sy, int64_t sz, double h,
                          double* u, const double* b, const int64_t* idx, int64_t count)
{
    og_grid g = og_make(dim, stencil, parity, nx, ny, nz, sy, sz, h);
    for (int64_t t = 0; t < count; ++t) og_update(&g, u, b, idx[t]);
}

/* nsweeps sweeps, each the colours 0..c-1 in order (Sec. 3, one loop over c). */
void og_gs_sweeps_f64(int dim, int stencil, int parity, int64_t nx, int64_t ny,
                      int64_t nz, int64_t sy, int64_t sz, double h,
                      double* u, const double* b, int nsweeps)
{
    int nc = og_num_colours(stencil, dim);
    for (int s = 0; s < nsweeps; ++s)
        for (int c = 0; c < nc; ++c)
            og_colour_pass_f64(dim, stencil, parity, nx, ny, nz, sy, sz, h, u, b, c);
}

void og_gs_sweeps_f32(int dim, int stencil, int parity, int64_t nx, int64_t ny,
                      int64_t nz, int64_t sy, int64_t sz, double h,
                      float* u, const float* b, int nsweeps)
{
    int nc = og_num_colours(stencil, dim);
    for (int s = 0; s < nsweeps; ++s)
        for (int c = 0; c < nc; ++c)
            og_colour_pass_f32(dim, stencil, parity, nx, ny, nz, sy, sz, h, u, b, c);
}

/* ------------------------------------------------------------------ */
/* Lexicographic Gauss-Seidel (the task-graph iterate of Sec. 3)        */
/* ------------------------------------------------------------------ */

/* Sec. 3's task graph keeps the issue order of the sequential loop: every
 * point is updated in place, z-y-x order with x innermost, from the newest
 * values of all its neighbours.  No colouring: a different iterate. */
void og_lex_sweeps_f64(int dim, int stencil, int parity, int64_t nx, int64_t ny,
                       int64_t nz, int64_t sy, int64_t sz, double h,
                       double* u, const double* b, int nsweeps)
{
    og_grid g = og_make(dim, stencil, parity, nx, ny, nz, sy, sz, h);
    for (int s = 0; s < nsweeps; ++s)
        for (int64_t k = 1; k <= g.nz; ++k)
            for (int64_t j = 1; j <= g.ny; ++j)
                for (int64_t i = 1; i <= g.nx; ++i)
                    og_update(&g, u, b, og_index(&g, i, j, k));
}

/* ------------------------------------------------------------------ */
/* Nested dissection (the other ordering of Sec. 3)                     */
/* ------------------------------------------------------------------ */

/* Sec. 3 splits the domain into 2^d blocks and a one-cell separator, recursively,
 * runs the blocks (which do not couple) before their separator, and leaves the
 * recursion depth and the order inside a separator to the machine.  Reading
 * taken here: a box whose every edge is at most `leaf` cells is a leaf and is
 * swept in z-y-x order; otherwise every axis longer than `leaf` is cut at the
 * cell lo + extent / 2, the sub-boxes (lower before upper half per axis, z
 * outermost) are processed recursively, then the separator -- the cells of the
 * box on a cut -- in z-y-x order.  Every cell is updated once per sweep, in
 * place: Gauss-Seidel in the dissection ordering, a different iterate from the
 * colouring. */
static void og_nd_box(const og_grid* g, double* u, const double* b, const int64_t* lo,
                      const int64_t* hi, int64_t leaf)
{
    int cut[3] = {0, 0, 0};
    int64_t m[3] = {0, 0, 0};
    int any = 0;
    for (int a = 0; a < g->dim; ++a) {
        const int64_t ext = hi[a] - lo[a] + 1;
        if (ext > leaf) {
            cut[a] = 1;
            m[a] = lo[a] + ext / 2;
            any = 1;
        }
    }
    if (any) {
        for (int hz = 0; hz <= cut[2]; ++hz)
            for (int hy = 0; hy <= cut[1]; ++hy)
                for (int hx = 0; hx <= cut[0]; ++hx) {
                    const int half[3] = {hx, hy, hz};
                    int64_t clo[3], chi[3];
                    int empty = 0;
                    for (int a = 0; a < 3; ++a) {
                        clo[a] = lo[a];
                        chi[a] = hi[a];
                        if (cut[a]) {
                            if (half[a] == 0) chi[a] = m[a] - 1;
                            else clo[a] = m[a] + 1;
                        }
                        if (clo[a] > chi[a]) empty = 1;
                    }
                    if (!empty) og_nd_box(g, u, b, clo, chi, leaf);
                }
    }
    for (int64_t k = lo[2]; k <= hi[2]; ++k)
        for (int64_t j = lo[1]; j <= hi[1]; ++j)
            for (int64_t i = lo[0]; i <= hi[0]; ++i) {
                const int on_cut = (cut[0] && i == m[0]) || (cut[1] && j == m[1]) || (cut[2] && k == m[2]);
                if (!any || on_cut) og_update(g, u, b, og_index(g, i, j, k));
            }
}

void og_nd_sweeps_f64(int dim, int stencil, int parity, int64_t nx, int64_t ny,
                      int64_t nz, int64_t sy, int64_t sz, double h,
                      double* u, const double* b, int nsweeps, int64_t leaf)
{
    og_grid g = og_make(dim, stencil, parity, nx, ny, nz, sy, sz, h);
    const int64_t lo[3] = {1, 1, 1}, hi[3] = {g.nx, g.ny, g.nz};
    for (int s = 0; s < nsweeps; ++s) og_nd_box(&g, u, b, lo, hi, leaf < 1 ? 1 : leaf);
}

void og_lex_sweeps_f32(int dim, int stencil, int parity, int64_t nx, int64_t ny,
                       int64_t nz, int64_t sy, int64_t sz, double h,
                       float* u, const float* b, int nsweeps)
{
    og_grid g = og_make(dim, stencil, parity, nx, ny, nz, sy, sz, h);
    for (int s = 0; s < nsweeps; ++s)
        for (int64_t k = 1; k <= g.nz; ++k)
            for (int64_t j = 1; j <= g.ny; ++j)
                for (int64_t i = 1; i <= g.nx; ++i)
                    og_update_f32(&g, u, b, og_index(&g, i, j, k));
}

/* ------------------------------------------------------------------ */
/* Expensive stencil evaluation S(k) (Sec. 2; load patterns of Sec. 4)  */
/* ------------------------------------------------------------------ */

/* Sec. 2 lets every stencil entry cost k floating-point operations; Sec. 4
 * realises it by adding k evaluations of sin to each prescribed entry, with k
 * either fixed or running linearly over the mesh.  Here the added terms are
 * z * sin(t a + j_o c), t = 1..k, with z = +0 and j_o = (oz+1)*9 + (oy+1)*3 +
 * (ox+1) the entry's index: each is a signed zero for finite arguments, so
 * S_o(k) == S_o exactly and the iterate is the k = 0 iterate, while the cost
 * grows with k. */
static double og_cost_entry(double w, int jo, int kq, double z, double a, double c)
{
    double s = w;
    for (int t = 1; t <= kq; ++t) s = s + z * sin((double)t * a + (double)jo * c);
    return s;
}

static void og_update_cost(const og_grid* g, double* u, const double* b, int64_t q, int kq,
                           double z, double a, double c)
{
    int zr = g->dim == 3 ? 1 : 0;
    double acc = 0.0;
    for (int oz = -zr; oz <= zr; ++oz)
        for (int oy = -1; oy <= 1; ++oy)
            for (int ox = -1; ox <= 1; ++ox) {
                if (ox == 0 && oy == 0 && oz == 0) continue;
                double w = og_weight(g->stencil, g->dim, ox, oy, oz);
                if (w == 0.0) continue;
                int jo = (oz + 1) * 9 + (oy + 1) * 3 + (ox + 1);
                acc = fma(og_cost_entry(w, jo, kq, z, a, c), u[q + oz * g->sz + oy * g->sy + ox], acc);
            }
    double w0 = og_weight(g->stencil, g->dim, 0, 0, 0);
    double x = (g->h * g->h * b[q] - acc) + (og_cost_entry(w0, 13, kq, z, a, c) - w0);
    u[q] = og_over_centre(g->stencil, g->dim, x);
}

/* nsweeps sweeps with S(k): k = kmax everywhere (hetero = 0) or
 * k = floor(kmax * l / N) over the lexicographic interior index l. */
void og_gs_sweeps_cost_f64(int dim, int stencil, int parity, int64_t nx, int64_t ny,
                           int64_t nz, int64_t sy, int64_t sz, double h,
                           double* u, const double* b, int nsweeps, int kmax, int hetero,
                           double z, double a, double c)
{
    og_grid g = og_make(dim, stencil, parity, nx, ny, nz, sy, sz, h);
    int nc = og_num_colours(stencil, dim);
    int64_t npts = g.nx * g.ny * g.nz;
    for (int s = 0; s < nsweeps; ++s)
        for (int col = 0; col < nc; ++col)
            for (int64_t k = 1; k <= g.nz; ++k)
                for (int64_t j = 1; j <= g.ny; ++j)
                    for (int64_t i = 1; i <= g.nx; ++i) {
                        if (og_colour(stencil, dim, parity, i, j, k) != col) continue;
                        int64_t l = ((k - 1) * g.ny + (j - 1)) * g.nx + (i - 1);
                        int kq = hetero ? (int)((int64_t)kmax * l / npts) : kmax;
                        og_update_cost(&g, u, b, og_index(&g, i, j, k), kq, z, a, c);
                    }
}

/* ------------------------------------------------------------------ */
/* Weighted Jacobi (separate output array)                              */
/* ------------------------------------------------------------------ */

/* tmp must have u's shape.  Its halo is overwritten with u's halo first; after
 * the call u holds the result (the last sweep's output is copied back when
 * the sweep count is odd). */
void og_jacobi_sweeps_f64(int dim, int stencil, int parity, int64_t nx, int64_t ny,
                          int64_t nz, int64_t sy, int64_t sz, double h,
                          double* u, const double* b, double* tmp, double omega,
                          int nsweeps, int64_t total_len)
{
    og_grid g = og_make(dim, stencil, parity, nx, ny, nz, sy, sz, h);
    double h2 = h * h;
    memcpy(tmp, u, (size_t)total_len * sizeof(double));
    double* src = u;
    double* dst = tmp;
    for (int s = 0; s < nsweeps; ++s) {
#pragma omp parallel for collapse(2) schedule(static)
        for (int64_t k = 1; k <= g.nz; ++k)
            for (int64_t j = 1; j <= g.ny; ++j)
                for (int64_t i = 1; i <= g.nx; ++i) {
                    int64_t q = og_index(&g, i, j, k);
                    double su = og_fullsum(&g, src, q);
                    dst[q] = fma(omega, og_over_centre(stencil, dim, h2 * b[q] - su), src[q]);
                }
        double* t = src; src = dst; dst = t;
    }
    if (src != u) memcpy(u, src, (size_t)total_len * sizeof(double));
}

void og_jacobi_sweeps_f32(int dim, int stencil, int parity, int64_t nx, int64_t ny,
                          int64_t nz, int64_t sy, int64_t sz, double h,
                          float* u, const float* b, float* tmp, double omega,
                          int nsweeps, int64_t total_len)
{
    og_grid g = og_make(dim, stencil, parity, nx, ny, nz, sy, sz, h);
    float h2 = (float)(h * h);
    float om = (float)omega;
    memcpy(tmp, u, (size_t)total_len * sizeof(float));
    float* src = u;
    float* dst = tmp;
    for (int s = 0; s < nsweeps; ++s) {
#pragma omp parallel for collapse(2) schedule(static)
        for (int64_t k = 1; k <= g.nz; ++k)
            for (int64_t j = 1; j <= g.ny; ++j)
                for (int64_t i = 1; i <= g.nx; ++i) {
                    int64_t q = og_index(&g, i, j, k);
                    float su = og_fullsum_f32(&g, src, q);
                    dst[q] = fmaf(om, og_over_centre_f32(stencil, dim, h2 * b[q] - su), src[q]);
                }
        float* t = src; src = dst; dst = t;
    }
    if (src != u) memcpy(u, src, (size_t)total_len * sizeof(float));
}

/* ------------------------------------------------------------------ */
/* Residual and norms                                                   */
/* ------------------------------------------------------------------ */

/* Neumaier's compensated summation: adds x into (*s, *c). */
static void og_neumaier(double* s, double* c, double x)
{
    double t = *s + x;
    if (fabs(*s) >= fabs(x)) *c += (*s - t) + x;
    else                     *c += (x - t) + *s;
    *s = t;
}

/* r = b - S u / h^2 over the interior (r may be NULL).  norms[0] = ||r||_2,
 * norms[1] = max |r|, norms[2] = ||b||_2, unweighted, interior points only. */
void og_residual_f64(int dim, int stencil, int parity, int64_t nx, int64_t ny,
                     int64_t nz, int64_t sy, int64_t sz, double h,
                     const double* u, const double* b, double* r, double* norms)
{
    og_grid g = og_make(dim, stencil, parity, nx, ny, nz, sy, sz, h);
    double h2 = h * h;
    double s_r = 0.0, c_r = 0.0, s_b = 0.0, c_b = 0.0, mx = 0.0;
    for (int64_t k = 1; k <= g.nz; ++k)
        for (int64_t j = 1; j <= g.ny; ++j)
            for (int64_t i = 1; i <= g.nx; ++i) {
                int64_t q = og_index(&g, i, j, k);
                double su = og_fullsum(&g, u, q);
                double rq = b[q] - su / h2;
                if (r) r[q] = rq;
                og_neumaier(&s_r, &c_r, rq * rq);
                og_neumaier(&s_b, &c_b, b[q] * b[q]);
                if (fabs(rq) > mx) mx = fabs(rq);
            }
    norms[0] = sqrt(s_r + c_r);
    norms[1] = mx;
    norms[2] = sqrt(s_b + c_b);
}

/* Residual of an FP32 grid, evaluated in FP64 from the stored binary32 values. */
void og_residual_f32in(int dim, int stencil, int parity, int64_t nx, int64_t ny,
                       int64_t nz, int64_t sy, int64_t sz, double h,
                       const float* u, const float* b, double* norms)
{
    og_grid g = og_make(dim, stencil, parity, nx, ny, nz, sy, sz, h);
    double h2 = h * h;
    double s_r = 0.0, c_r = 0.0, s_b = 0.0, c_b = 0.0, mx = 0.0;
    int zr = dim == 3 ? 1 : 0;
    for (int64_t k = 1; k <= g.nz; ++k)
        for (int64_t j = 1; j <= g.ny; ++j)
            for (int64_t i = 1; i <= g.nx; ++i) {
                int64_t q = og_index(&g, i, j, k);
                double su = 0.0;
                for (int oz = -zr; oz <= zr; ++oz)
                    for (int oy = -1; oy <= 1; ++oy)
                        for (int ox = -1; ox <= 1; ++ox) {
                            double w = og_weight(stencil, dim, ox, oy, oz);
                            if (w == 0.0) continue;
                            su = fma(w, (double)u[q + oz * g.sz + oy * g.sy + ox], su);
                        }
                double bq = (double)b[q];
                double rq = bq - su / h2;
                og_neumaier(&s_r, &c_r, rq * rq);
                og_neumaier(&s_b, &c_b, bq * bq);
                if (fabs(rq) > mx) mx = fabs(rq);
            }
    norms[0] = sqrt(s_r + c_r);
    norms[1] = mx;
    norms[2] = sqrt(s_b + c_b);
}

/* ------------------------------------------------------------------ */
/* Second formulation of the Q1 operator: element by element            */
/* ------------------------------------------------------------------ */

/* Reference-element stiffness of the d-linear element on the unit cell,
 * entry for two vertices that differ in `ndiff` coordinates:
 *   d = 2: 2/3, -1/6, -1/3          (ndiff = 0, 1, 2)
 *   d = 3: 1/3, 0, -1/12, -1/12     (ndiff = 0, 1, 2, 3)                    */
double og_q1_kref(int dim, int ndiff)
{
    if (dim == 2) {
        if (ndiff == 0) return 2.0 / 3.0;
        if (ndiff == 1) return -1.0 / 6.0;
        return -1.0 / 3.0;
    }
    if (ndiff == 0) return 1.0 / 3.0;
    if (ndiff == 1) return 0.0;
    return -1.0 / 12.0;
}

/* out_q = (S u)_q for every interior vertex q, accumulated cell by cell:
 * each cell (one per index box [i,i+1]x[j,j+1](x[k,k+1]) touching the
 * interior) adds K_ref u_e into its 2^d vertices.  out must be zero on entry
 * (halo entries of out receive partial sums and are not meaningful). */
void og_q1_apply_cellwise(int dim, int64_t nx, int64_t ny, int64_t nz,
                          int64_t sy, int64_t sz, const double* u, double* out)
{
    int nv = 1 << dim;
    int64_t kz = dim == 3 ? nz : 0;
    for (int64_t k = 0; k <= kz; ++k)
        for (int64_t j = 0; j <= ny; ++j)
            for (int64_t i = 0; i <= nx; ++i) {
                for (int a = 0; a < nv; ++a) {
                    int64_t qa = (i + (a & 1)) + (j + ((a >> 1) & 1)) * sy
                               + (dim == 3 ? (k + ((a >> 2) & 1)) * sz : 0);
                    double acc = 0.0;
                    for (int bb = 0; bb < nv; ++bb) {
                        int64_t qb = (i + (bb & 1)) + (j + ((bb >> 1) & 1)) * sy
                                   + (dim == 3 ? (k + ((bb >> 2) & 1)) * sz : 0);
                        int x = a ^ bb;
                        int ndiff = (x & 1) + ((x >> 1) & 1) + ((x >> 2) & 1);
                        double kab = og_q1_kref(dim, ndiff);
                        if (kab == 0.0) continue;
                        acc += kab * u[qb];
                    }
                    out[qa] += acc;
                }
            }
}

/* The same cell-wise accumulation in 2^d cell-colour passes: colour of the
 * cell with lower corner (i, j, k) = (i mod 2) + 2 (j mod 2) + 4 (k mod 2);
 * cells of one colour share no vertex, so a pass has no write conflict (the
 * race-free accumulation into vertices by cell colouring).  Colours 0..2^d-1
 * in order, z-y-x within a colour; each vertex therefore receives its 2^d
 * contributions in colour order. */
void og_q1_apply_cellwise_coloured(int dim, int64_t nx, int64_t ny, int64_t nz,
                                   int64_t sy, int64_t sz, const double* u, double* out)
{
    int nv = 1 << dim;
    int64_t kz = dim == 3 ? nz : 0;
    for (int col = 0; col < nv; ++col)
        for (int64_t k = 0; k <= kz; ++k)
            for (int64_t j = 0; j <= ny; ++j)
                for (int64_t i = 0; i <= nx; ++i) {
                    int cc = (int)(i & 1) + 2 * (int)(j & 1) + (dim == 3 ? 4 * (int)(k & 1) : 0);
                    if (cc != col) continue;
                    for (int a = 0; a < nv; ++a) {
                        int64_t qa = (i + (a & 1)) + (j + ((a >> 1) & 1)) * sy
                                   + (dim == 3 ? (k + ((a >> 2) & 1)) * sz : 0);
                        double acc = 0.0;
                        for (int bb = 0; bb < nv; ++bb) {
                            int64_t qb = (i + (bb & 1)) + (j + ((bb >> 1) & 1)) * sy
                                       + (dim == 3 ? (k + ((bb >> 2) & 1)) * sz : 0);
                            int x = a ^ bb;
                            int ndiff = (x & 1) + ((x >> 1) & 1) + ((x >> 2) & 1);
                            double kab = og_q1_kref(dim, ndiff);
                            if (kab == 0.0) continue;
                            acc += kab * u[qb];
                        }
                        out[qa] += acc;
                    }
                }
}

/* (S u)_q by the stencil form, for comparison with the cell-wise form. */
void og_apply_stencil(int dim, int stencil, int64_t nx, int64_t ny, int64_t nz,
                      int64_t sy, int64_t sz, const double* u, double* out)
{
    og_grid g = og_make(dim, stencil, 0, nx, ny, nz, sy, sz, 1.0);
    for (int64_t k = 1; k <= g.nz; ++k)
        for (int64_t j = 1; j <= g.ny; ++j)
            for (int64_t i = 1; i <= g.nx; ++i) {
                int64_t q = og_index(&g, i, j, k);
                out[q] = og_fullsum(&g, u, q);
            }
}

/* ------------------------------------------------------------------ */
/* Grid transfers of a geometric multigrid V-cycle                       */
/* ------------------------------------------------------------------ */
/* The paper names multigrid as the setting its smoothers serve (Sec. 1); a
 * V-cycle here uses the coloured Gauss-Seidel sweep above as its smoother and
 * the textbook vertex-centred transfers below.  A fine grid has n_f = 2 n_c + 1
 * interior points per axis, and fine index i = 2 I lies on coarse index I, so
 * the coarse halo (I = 0, n_c + 1) lies on the fine halo.
 *
 * Restriction by full weighting, at every coarse interior point:
 *   bc_I = sum over o in {-1,0,1}^d of w(o_x) w(o_y) [w(o_z)] r_{2I+o},
 *   w(0) = 1/2, w(+-1) = 1/4 (weights sum to 1; R = P^T / 2^d),
 * terms in lexicographic (oz, oy, ox) order, each added with one fma; the
 * coarse iterate uc is set to zero at the same points.
 *
 * Prolongation by d-linear interpolation, added to the fine iterate at every
 * fine interior point:
 *   uf_i <- uf_i + sum over coarse c with |2 c_m - i_m| <= 1 for every axis m
 *           of prod_m (1 if 2 c_m = i_m, else 1/2) uc_c,
 * coarse halo values included, terms in increasing (cz, cy, cx) order, each
 * added with one fma, then one addition to uf.  All weights are powers of two,
 * so their products are exact.                                              */
static double og_fw(int o) { return o == 0 ? 0.5 : 0.25; }

void og_restrict_f64(int dim, int64_t nxc, int64_t nyc, int64_t nzc, int64_t syc, int64_t szc,
                     int64_t syf, int64_t szf, const double* r, double* bc, double* uc)
{
    int zr = dim == 3 ? 1 : 0;
    int64_t nz = dim == 3 ? nzc : 1;
    for (int64_t K = 1; K <= nz; ++K)
        for (int64_t J = 1; J <= nyc; ++J)
            for (int64_t I = 1; I <= nxc; ++I) {
                int64_t qf = (dim == 3 ? 2 * K * szf : 0) + 2 * J * syf + 2 * I;
                double acc = 0.0;
                for (int oz = -zr; oz <= zr; ++oz)
                    for (int oy = -1; oy <= 1; ++oy)
                        for (int ox = -1; ox <= 1; ++ox) {
                            double w = (dim == 3 ? og_fw(oz) : 1.0) * og_fw(oy) * og_fw(ox);
                            acc = fma(w, r[qf + oz * szf + oy * syf + ox], acc);
                        }
                int64_t qc = (dim == 3 ? K * szc : 0) + J * syc + I;
                bc[qc] = acc;
                uc[qc] = 0.0;
            }
}

void og_prolong_add_f64(int dim, int64_t nxf, int64_t nyf, int64_t nzf, int64_t syf, int64_t szf,
                        int64_t syc, int64_t szc, const double* uc, double* uf)
{
    int64_t nz = dim == 3 ? nzf : 1;
    for (int64_t k = 1; k <= nz; ++k)
        for (int64_t j = 1; j <= nyf; ++j)
            for (int64_t i = 1; i <= nxf; ++i) {
                /* coarse neighbours along an axis: t/2, and t/2 + 1 when t is odd */
                int nkz = dim == 3 ? 1 + (int)(k & 1) : 1;
                int nky = 1 + (int)(j & 1), nkx = 1 + (int)(i & 1);
                double wz = dim == 3 && (k & 1) ? 0.5 : 1.0;
                double wy = (j & 1) ? 0.5 : 1.0, wx = (i & 1) ? 0.5 : 1.0;
                double acc = 0.0;
                for (int a = 0; a < nkz; ++a)
                    for (int bb = 0; bb < nky; ++bb)
                        for (int c = 0; c < nkx; ++c) {
                            int64_t qc = (dim == 3 ? (k / 2 + a) * szc : 0) + (j / 2 + bb) * syc + i / 2 + c;
                            acc = fma(wz * wy * wx, uc[qc], acc);
                        }
                int64_t q = (dim == 3 ? k * szf : 0) + j * syf + i;
                uf[q] = uf[q] + acc;
            }
}
