// Basic kernels: one launch per colour pass, weighted Jacobi, halo and
// interior copies, and the residual with a deterministic two-stage reduction.
//
// The colour pass is the GPU form of the paper's flat BSP colouring (Sec. 3:
// one loop over the c colours, each pass a parallel loop over the grid, a
// global synchronisation between passes): here one kernel launch per colour,
// the stream order being the synchronisation.  Only the points of the colour
// are enumerated, x fastest within a wavefront.
#include "cs_device.h"
#include "cs_internal.h"

#include <stdint.h>

namespace cs {

namespace {

constexpr int kBX = 64;  // threads along x (one wavefront)
constexpr int kBY = 4;   // rows per block

// Number of i in [i0, n] with step 2.
__host__ __device__ inline int64_t count_step2(int64_t i0, int64_t n)
{
    return i0 <= n ? (n - i0) / 2 + 1 : 0;
}

__device__ __forceinline__ double sin_t(double x) { return sin(x); }
__device__ __forceinline__ float sin_t(float x) { return sinf(x); }

// Expensive stencil evaluation S(k) (Sec. 2 and Sec. 4): every nonzero entry
// S_o used by an update is recomputed as S_o + sum_{t=1..k} zero * sin(t a + j_o c)
// with j_o the entry's index and zero = +0, a, c run-time arguments.  For
// finite arguments every added term is a signed zero, so S_o(k) equals S_o bit
// for bit and the iterate is the k = 0 iterate, while each entry costs k sin
// evaluations.  hetero: k = floor(kmax * l / N) over the lexicographic
// interior index l (the load runs linearly over the mesh), else k = kmax.
template <typename T>
__device__ __forceinline__ T costly_entry(T w, int jo, int kq, T zero, T a, T c)
{
    T s = w;
    for (int t = 1; t <= kq; ++t) s = s + zero * sin_t(T(t) * a + T(jo) * c);
    return s;
}

template <typename T, int DIM, int ST, bool COST>
__global__ void __launch_bounds__(kBX* kBY)
k_colour_pass(T* __restrict__ u, const T* __restrict__ b, Geo g, T h2, int colour,
              int64_t rows_y, int64_t rows_z, int64_t xblocks, StencilCost cost)
{
    // With a load that grows along the mesh, the blocks are taken in reverse
    // order: the dearest rows start first and the cheap ones fill in behind
    // them (longest-first list scheduling by the hardware dispatcher).
    const int64_t bid = (COST && cost.hetero) ? (int64_t)gridDim.x - 1 - blockIdx.x : blockIdx.x;
    const int64_t xb = bid % xblocks;
    const int64_t row = (bid / xblocks) * kBY + threadIdx.y;
    if (row >= rows_y * rows_z) return;
    const int64_t ty = row % rows_y;
    const int64_t tz = row / rows_y;
    int64_t i0, j, k;
    if (ST == FD) {
        j = 1 + ty;
        k = 1 + tz;
        const int64_t kk = DIM == 3 ? k - 1 : 0;
        i0 = 1 + ((colour + (j - 1) + kk + g.parity) & 1);
    } else {
        const int px = colour & 1, py = (colour >> 1) & 1, pz = (colour >> 2) & 1;
        i0 = 1 + ((px + g.parity) & 1);
        j = 1 + ((py + g.parity) & 1) + 2 * ty;
        k = DIM == 3 ? 1 + ((pz + g.parity) & 1) + 2 * tz : 1;
    }
    const int64_t i = i0 + 2 * (xb * kBX + threadIdx.x);
    if (i > g.nx) return;
    const int64_t q = (DIM == 3 ? k * g.sz : 0) + j * g.sy + i;
    const int64_t sy = g.sy, sz = g.sz;
    auto ld = [&](int ox, int oy, int oz) { return u[q + oz * sz + oy * sy + ox]; };
    if (!COST) {
        u[q] = gs_value<T, DIM, ST>(h2, b[q], ld);
        return;
    }
    int kq = cost.kmax;
    if (cost.hetero) {
        const int64_t l = ((DIM == 3 ? (k - 1) * g.ny : 0) + (j - 1)) * g.nx + (i - 1);
        kq = (int)((int64_t)cost.kmax * l / cost.npts);
    }
    const T zero = (T)cost.zero, a = (T)cost.a, c = (T)cost.c;
    // the ordered sum of gs_value with run-time entries S_o(k) == S_o
    T acc = T(0);
#pragma unroll
    for (int oz = (DIM == 3 ? -1 : 0); oz <= (DIM == 3 ? 1 : 0); ++oz)
#pragma unroll
        for (int oy = -1; oy <= 1; ++oy)
#pragma unroll
            for (int ox = -1; ox <= 1; ++ox) {
                if (ox == 0 && oy == 0 && oz == 0) continue;
                const T w = weight<T, DIM, ST>(ox, oy, oz);
                if (w == T(0)) continue;
                const int jo = (oz + 1) * 9 + (oy + 1) * 3 + (ox + 1);
                acc = fma_t(costly_entry(w, jo, kq, zero, a, c), ld(ox, oy, oz), acc);
            }
    const T w0 = weight<T, DIM, ST>(0, 0, 0);
    const T x = (h2 * b[q] - acc) + (costly_entry(w0, 13, kq, zero, a, c) - w0);
    u[q] = over_centre<T, DIM, ST>(x);
}

// Lexicographic Gauss-Seidel by hyperplane wavefronts (the task-graph
// iterate of Sec. 3).  With hyperplane index s = i + wj j + wk k, every
// neighbour that precedes a point in the natural (z, y, x) order lies on a
// smaller s and every later one on a larger s: (wj, wk) = (1, 1) for the
// 2d+1-point stencils, (2, 4) for the 3^d-point ones (an offset (1, -1, 0)
// precedes, 1 - wj < 0; (1, 1, -1) precedes, 1 + wj - wk < 0).  So the points
// of one hyperplane are independent and one launch per s, in increasing s,
// reproduces the sequential sweep.  One thread per (j, k); i follows.
template <typename T, int DIM, int ST>
__global__ void __launch_bounds__(256)
k_lex_plane(T* __restrict__ u, const T* __restrict__ b, Geo g, T h2, int64_t s, int64_t k_lo,
            int64_t nk)
{
    constexpr int64_t WJ = ST == FD ? 1 : 2, WK = ST == FD ? 1 : 4;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= g.ny * nk) return;
    const int64_t j = 1 + t % g.ny;
    const int64_t k = DIM == 3 ? k_lo + t / g.ny : 1;
    const int64_t i = s - WJ * j - (DIM == 3 ? WK * k : 0);
    if (i < 1 || i > g.nx) return;
    const int64_t q = (DIM == 3 ? k * g.sz : 0) + j * g.sy + i;
    const int64_t sy = g.sy, sz = g.sz;
    auto ld = [&](int ox, int oy, int oz) { return u[q + oz * sz + oy * sy + ox]; };
    u[q] = gs_value<T, DIM, ST>(h2, b[q], ld);
}

template <typename T, int DIM, int ST>
__global__ void __launch_bounds__(kBX* kBY)
k_jacobi(const T* __restrict__ src, T* __restrict__ dst, const T* __restrict__ b, Geo g, T h2,
         T omega, int64_t xblocks)
{
    const int64_t bid = blockIdx.x;
    const int64_t xb = bid % xblocks;
    const int64_t row = (bid / xblocks) * kBY + threadIdx.y;
    if (row >= g.ny * g.nz) return;
    const int64_t j = 1 + row % g.ny;
    const int64_t k = 1 + row / g.ny;
    const int64_t i = 1 + xb * kBX + threadIdx.x;
    if (i > g.nx) return;
    const int64_t q = (DIM == 3 ? k * g.sz : 0) + j * g.sy + i;
    const int64_t sy = g.sy, sz = g.sz;
    auto ld = [&](int ox, int oy, int oz) { return src[q + oz * sz + oy * sy + ox]; };
    dst[q] = jacobi_value<T, DIM, ST>(h2, omega, b[q], src[q], ld);
}

// Seeded uniform[-1, 1) field on the interior: SplitMix64 in counter form,
// value(seed, l) = mix64(seed + (l + 1) * 0x9E3779B97F4A7C15) over the
// lexicographic interior index l (x fastest), (v >> 11) * 2^-52 - 1 exact in
// binary64 (rounded to T).  The same published generator as the host-side
// input module, so device and host fields agree bit for bit.
__device__ __forceinline__ uint64_t splitmix_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

template <typename T, int DIM>
__global__ void __launch_bounds__(256)
k_fill_uniform(T* __restrict__ a, Geo g, uint64_t seed)
{
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= g.nx * g.ny * g.nz) return;
    const int64_t i = 1 + l % g.nx, j = 1 + (l / g.nx) % g.ny, k = 1 + l / (g.nx * g.ny);
    const uint64_t v = splitmix_mix(seed + ((uint64_t)l + 1) * 0x9E3779B97F4A7C15ull);
    const double x = (double)(v >> 11) * 0x1p-52 - 1.0;
    a[(DIM == 3 ? k * g.sz : 0) + j * g.sy + i] = (T)x;
}

// Operator application y = A u = (S u) / h^2 at interior points (the
// separate-output-array mat-vec of Sec. 2), stencil form: the full ordered
// sum of the plain definition.
template <typename T, int DIM, int ST>
__global__ void __launch_bounds__(kBX* kBY)
k_apply(const T* __restrict__ u, T* __restrict__ y, Geo g, T h2, int64_t xblocks)
{
    const int64_t bid = blockIdx.x;
    const int64_t xb = bid % xblocks;
    const int64_t row = (bid / xblocks) * kBY + threadIdx.y;
    if (row >= g.ny * g.nz) return;
    const int64_t j = 1 + row % g.ny;
    const int64_t k = 1 + row / g.ny;
    const int64_t i = 1 + xb * kBX + threadIdx.x;
    if (i > g.nx) return;
    const int64_t q = (DIM == 3 ? k * g.sz : 0) + j * g.sy + i;
    const int64_t sy = g.sy, sz = g.sz;
    auto ld = [&](int ox, int oy, int oz) { return u[q + oz * sz + oy * sy + ox]; };
    y[q] = ordered_sum<T, DIM, ST, true>(ld) / h2;
}

// The d-linear operator applied element by element ("cell-wise, accumulating
// into vertices"): every cell with lower corner (i, j, k), 0 <= i <= nx etc.,
// adds K_ref u_e into its 2^d vertices, K_ref the assembled d-linear element
// stiffness (entries by the number of coordinates in which two vertices
// differ: 2D 2/3, -1/6, -1/3; 3D 1/3, 0, -1/12, -1/12).  Cells are taken in
// 2^d colour passes, colour = parities of the lower corner; cells of one
// colour share no vertex, so each pass scatters without conflicts and every
// vertex receives its contributions in colour order.  One thread per cell.
template <typename T, int DIM>
__device__ __forceinline__ T kref(int ndiff)
{
    if (DIM == 2) return ndiff == 0 ? T(2) / T(3) : (ndiff == 1 ? T(-1) / T(6) : T(-1) / T(3));
    return ndiff == 0 ? T(1) / T(3) : (ndiff == 1 ? T(0) : T(-1) / T(12));
}

template <typename T, int DIM>
__global__ void __launch_bounds__(256)
k_cell_pass(const T* __restrict__ u, T* __restrict__ y, Geo g, int colour, int64_t cx, int64_t cy,
            int64_t cz)
{
    constexpr int NV = 1 << DIM;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= cx * cy * cz) return;
    const int64_t i = (colour & 1) + 2 * (t % cx);
    const int64_t j = ((colour >> 1) & 1) + 2 * ((t / cx) % cy);
    const int64_t k = DIM == 3 ? ((colour >> 2) & 1) + 2 * (t / (cx * cy)) : 0;
    const int64_t base = (DIM == 3 ? k * g.sz : 0) + j * g.sy + i;
    int64_t off[NV];
    T ue[NV];
#pragma unroll
    for (int a = 0; a < NV; ++a) {
        off[a] = base + (a & 1) + ((a >> 1) & 1) * g.sy + (DIM == 3 ? ((a >> 2) & 1) * g.sz : 0);
        ue[a] = u[off[a]];
    }
#pragma unroll
    for (int a = 0; a < NV; ++a) {
        T acc = T(0);
#pragma unroll
        for (int bb = 0; bb < NV; ++bb) {
            const int x = a ^ bb;
            const T kab = kref<T, DIM>((x & 1) + ((x >> 1) & 1) + ((x >> 2) & 1));
            if (kab == T(0)) continue;
            acc = acc + kab * ue[bb];
        }
        y[off[a]] = y[off[a]] + acc;
    }
}

// y over the whole halo'd extent (the cell passes write partial sums into
// the halo vertices too) set to zero, or the interior divided by h^2.
template <typename T, int DIM>
__global__ void __launch_bounds__(256)
k_fill_or_scale(T* __restrict__ y, Geo g, T h2, int scale)
{
    const int64_t wx = g.nx + 2, wy = g.ny + 2;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= wx * wy * (DIM == 3 ? g.nz + 2 : 1)) return;
    const int64_t i = t % wx, j = (t / wx) % wy, k = DIM == 3 ? t / (wx * wy) : 0;
    const int64_t q = (DIM == 3 ? k * g.sz : 0) + j * g.sy + i;
    if (!scale) {
        y[q] = T(0);
        return;
    }
    const bool inner = i >= 1 && i <= g.nx && j >= 1 && j <= g.ny && (DIM == 2 || (k >= 1 && k <= g.nz));
    if (inner) y[q] = y[q] / h2;
}

// Halo points enumerated as: (3D) planes k = 0 and k = nz+1 in full, then for
// each interior plane the rows j = 0, j = ny+1 and the columns i = 0, i = nx+1.
template <typename T, int DIM>
__global__ void __launch_bounds__(256)
k_halo_copy(const T* __restrict__ src, T* __restrict__ dst, Geo g, int64_t total)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const int64_t wx = g.nx + 2;
    const int64_t plane = wx * (g.ny + 2);
    int64_t i, j, k;
    int64_t r = t;
    if (DIM == 3 && r < 2 * plane) {
        k = r < plane ? 0 : g.nz + 1;
        r %= plane;
        j = r / wx;
        i = r % wx;
    } else {
        if (DIM == 3) r -= 2 * plane;
        const int64_t per = 2 * wx + 2 * g.ny;
        k = DIM == 3 ? 1 + r / per : 0;
        r %= per;
        if (r < 2 * wx) {
            j = r < wx ? 0 : g.ny + 1;
            i = r % wx;
        } else {
            r -= 2 * wx;
            j = 1 + r / 2;
            i = (r & 1) ? g.nx + 1 : 0;
        }
    }
    const int64_t q = (DIM == 3 ? k * g.sz : 0) + j * g.sy + i;
    dst[q] = src[q];
}

template <typename T, int DIM>
__global__ void __launch_bounds__(kBX* kBY)
k_interior_copy(const T* __restrict__ src, T* __restrict__ dst, Geo g, int64_t xblocks)
{
    const int64_t bid = blockIdx.x;
    const int64_t xb = bid % xblocks;
    const int64_t row = (bid / xblocks) * kBY + threadIdx.y;
    if (row >= g.ny * g.nz) return;
    const int64_t j = 1 + row % g.ny;
    const int64_t k = 1 + row / g.ny;
    const int64_t i = 1 + xb * kBX + threadIdx.x;
    if (i > g.nx) return;
    const int64_t q = (DIM == 3 ? k * g.sz : 0) + j * g.sy + i;
    dst[q] = src[q];
}

// Fixed-shape tree reduction of three values over a 256-thread block.
__device__ inline void block_reduce3(double& a, double& m, double& c, double* sh)
{
    const int t = threadIdx.y * blockDim.x + threadIdx.x;
    sh[t] = a;
    sh[256 + t] = m;
    sh[512 + t] = c;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) {
            sh[t] = sh[t] + sh[t + w];
            sh[256 + t] = fmax(sh[256 + t], sh[256 + t + w]);
            sh[512 + t] = sh[512 + t] + sh[512 + t + w];
        }
        __syncthreads();
    }
    a = sh[0];
    m = sh[256];
    c = sh[512];
}

// Stage 1: each block walks a fixed set of (x-block, row-group) tiles.
template <typename S, int DIM, int ST>
__global__ void __launch_bounds__(kBX* kBY)
k_residual(const S* __restrict__ u, const S* __restrict__ b, S* __restrict__ r, Geo g,
           double h2, int64_t xblocks, int64_t tiles, Partial* __restrict__ partials)
{
    __shared__ double sh[3 * 256];
    double s_r2 = 0.0, mx = 0.0, s_b2 = 0.0;
    const int64_t sy = g.sy, sz = g.sz;
    for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const int64_t xb = tile % xblocks;
        const int64_t row = (tile / xblocks) * kBY + threadIdx.y;
        const int64_t i = 1 + xb * kBX + threadIdx.x;
        if (row >= g.ny * g.nz || i > g.nx) continue;
        const int64_t j = 1 + row % g.ny;
        const int64_t k = 1 + row / g.ny;
        const int64_t q = (DIM == 3 ? k * g.sz : 0) + j * g.sy + i;
        auto ld = [&](int ox, int oy, int oz) { return (double)u[q + oz * sz + oy * sy + ox]; };
        const double su = ordered_sum<double, DIM, ST, true>(ld);
        const double bq = (double)b[q];
        const double rq = bq - su / h2;
        if (r) r[q] = (S)rq;
        s_r2 += rq * rq;
        s_b2 += bq * bq;
        mx = fmax(mx, fabs(rq));
    }
    block_reduce3(s_r2, mx, s_b2, sh);
    if (threadIdx.x == 0 && threadIdx.y == 0) {
        partials[blockIdx.x].sum_r2 = s_r2;
        partials[blockIdx.x].max_r = mx;
        partials[blockIdx.x].sum_b2 = s_b2;
    }
}

// Residual of an FP64 grid with the scaled FP32 copy r32 = fl32(r * inv_scale)
// and e32 = 0 written at the same points of the FP32 layout g2 (2D grids and
// grids the streaming kernel does not cover).
template <int DIM, int ST>
__global__ void __launch_bounds__(kBX* kBY)
k_ir_residual(const double* __restrict__ u, const double* __restrict__ b, Geo g, double h2,
              double inv_scale, Geo g2, float* __restrict__ r32, float* __restrict__ e32,
              int64_t xblocks, int64_t tiles, Partial* __restrict__ partials)
{
    __shared__ double sh[3 * 256];
    double s_r2 = 0.0, mx = 0.0, s_b2 = 0.0;
    const int64_t sy = g.sy, sz = g.sz;
    for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const int64_t xb = tile % xblocks;
        const int64_t row = (tile / xblocks) * kBY + threadIdx.y;
        const int64_t i = 1 + xb * kBX + threadIdx.x;
        if (row >= g.ny * g.nz || i > g.nx) continue;
        const int64_t j = 1 + row % g.ny;
        const int64_t k = 1 + row / g.ny;
        const int64_t q = (DIM == 3 ? k * g.sz : 0) + j * g.sy + i;
        const int64_t q2 = (DIM == 3 ? k * g2.sz : 0) + j * g2.sy + i;
        auto ld = [&](int ox, int oy, int oz) { return u[q + oz * sz + oy * sy + ox]; };
        const double su = ordered_sum<double, DIM, ST, true>(ld);
        const double bq = b[q];
        const double rq = bq - su / h2;
        r32[q2] = (float)(rq * inv_scale);
        e32[q2] = 0.0f;
        s_r2 += rq * rq;
        s_b2 += bq * bq;
        mx = fmax(mx, fabs(rq));
    }
    block_reduce3(s_r2, mx, s_b2, sh);
    if (threadIdx.x == 0 && threadIdx.y == 0) {
        partials[blockIdx.x].sum_r2 = s_r2;
        partials[blockIdx.x].max_r = mx;
        partials[blockIdx.x].sum_b2 = s_b2;
    }
}

// x <- x + e32 * scale (FP64) over the interior; scale is a power of two.
template <int DIM>
__global__ void __launch_bounds__(kBX* kBY)
k_ir_update(double* __restrict__ x, Geo g, const float* __restrict__ e32, Geo g2, double scale,
            int64_t xblocks)
{
    const int64_t bid = blockIdx.x;
    const int64_t xb = bid % xblocks;
    const int64_t row = (bid / xblocks) * kBY + threadIdx.y;
    if (row >= g.ny * g.nz) return;
    const int64_t j = 1 + row % g.ny;
    const int64_t k = 1 + row / g.ny;
    const int64_t i = 1 + xb * kBX + threadIdx.x;
    if (i > g.nx) return;
    const int64_t q = (DIM == 3 ? k * g.sz : 0) + j * g.sy + i;
    const int64_t q2 = (DIM == 3 ? k * g2.sz : 0) + j * g2.sy + i;
    x[q] = x[q] + (double)e32[q2] * scale;
}

// Stage 2: one block folds the partials in a fixed order.
__global__ void __launch_bounds__(256)
k_residual_finish(const Partial* __restrict__ partials, int count, double* __restrict__ norms)
{
    __shared__ double sh[3 * 256];
    double a = 0.0, m = 0.0, c = 0.0;
    for (int p = threadIdx.x; p < count; p += 256) {
        a += partials[p].sum_r2;
        m = fmax(m, partials[p].max_r);
        c += partials[p].sum_b2;
    }
    block_reduce3(a, m, c, sh);
    if (threadIdx.x == 0) {
        norms[0] = sqrt(a);
        norms[1] = m;
        norms[2] = sqrt(c);
    }
}

template <typename T, int DIM, int ST>
cs_status colour_pass_t(const Geo& g, void* u, const void* b, double h2, int colour,
                        const StencilCost* cost, hipStream_t s)
{
    int64_t rows_y, rows_z, xcount;
    if (ST == FD) {
        rows_y = g.ny;
        rows_z = DIM == 3 ? g.nz : 1;
        xcount = (g.nx + 1) / 2;
    } else {
        const int px = colour & 1, py = (colour >> 1) & 1, pz = (colour >> 2) & 1;
        xcount = count_step2(1 + ((px + g.parity) & 1), g.nx);
        rows_y = count_step2(1 + ((py + g.parity) & 1), g.ny);
        rows_z = DIM == 3 ? count_step2(1 + ((pz + g.parity) & 1), g.nz) : 1;
    }
    if (xcount == 0 || rows_y == 0 || rows_z == 0) return CS_OK;
    const int64_t xblocks = (xcount + kBX - 1) / kBX;
    const int64_t rblocks = (rows_y * rows_z + kBY - 1) / kBY;
    const int64_t blocks = xblocks * rblocks;
    if (blocks > 0x7fffffff) {
        set_error("colour pass: grid too large (%lld blocks)", (long long)blocks);
        return CS_EUNSUPPORTED;
    }
    if (cost)
        hipLaunchKernelGGL((k_colour_pass<T, DIM, ST, true>), dim3((unsigned)blocks),
                           dim3(kBX, kBY), 0, s, (T*)u, (const T*)b, g, (T)h2, colour, rows_y,
                           rows_z, xblocks, *cost);
    else
        hipLaunchKernelGGL((k_colour_pass<T, DIM, ST, false>), dim3((unsigned)blocks),
                           dim3(kBX, kBY), 0, s, (T*)u, (const T*)b, g, (T)h2, colour, rows_y,
                           rows_z, xblocks, StencilCost{});
    return check_launch("colour pass");
}

template <typename T, int DIM, int ST>
cs_status lex_sweep_t(const Geo& g, void* u, const void* b, double h2, hipStream_t s)
{
    const int64_t wj = ST == FD ? 1 : 2, wk = ST == FD ? 1 : 4;
    const int64_t s_lo = 1 + wj + (DIM == 3 ? wk : 0);
    const int64_t s_hi = g.nx + wj * g.ny + (DIM == 3 ? wk * g.nz : 0);
    for (int64_t sp = s_lo; sp <= s_hi; ++sp) {
        // planes k with some i in [1, nx] and j in [1, ny] on this hyperplane
        int64_t k_lo = 1, k_hi = 1;
        if (DIM == 3) {
            const int64_t r_hi = sp - 1 - wj;              // wk k <= s - 1 - wj
            const int64_t r_lo = sp - g.nx - wj * g.ny;    // wk k >= s - nx - wj ny
            k_hi = r_hi / wk;
            k_lo = r_lo <= wk ? 1 : (r_lo + wk - 1) / wk;
            if (k_hi > g.nz) k_hi = g.nz;
            if (k_lo > k_hi) continue;
        }
        const int64_t nk = k_hi - k_lo + 1;
        const int64_t threads = g.ny * nk;
        const int64_t blocks = (threads + 255) / 256;
        if (blocks > 0x7fffffff) {
            set_error("lexicographic sweep: grid too large");
            return CS_EUNSUPPORTED;
        }
        hipLaunchKernelGGL((k_lex_plane<T, DIM, ST>), dim3((unsigned)blocks), dim3(256), 0, s,
                           (T*)u, (const T*)b, g, (T)h2, sp, k_lo, nk);
    }
    return check_launch("lexicographic sweep");
}

template <typename T, int DIM, int ST>
cs_status jacobi_t(const Geo& g, const void* src, void* dst, const void* b, double h2,
                   double omega, hipStream_t s)
{
    const int64_t xblocks = (g.nx + kBX - 1) / kBX;
    const int64_t blocks = xblocks * ((g.ny * g.nz + kBY - 1) / kBY);
    if (blocks > 0x7fffffff) {
        set_error("jacobi: grid too large");
        return CS_EUNSUPPORTED;
    }
    hipLaunchKernelGGL((k_jacobi<T, DIM, ST>), dim3((unsigned)blocks), dim3(kBX, kBY), 0, s,
                       (const T*)src, (T*)dst, (const T*)b, g, (T)h2, (T)omega, xblocks);
    return check_launch("jacobi");
}

template <typename S, int DIM, int ST>
cs_status residual_t(const Geo& g, const void* u, const void* b, void* r, double h2,
                     Partial* partials, double* norms, hipStream_t s)
{
    const int64_t xblocks = (g.nx + kBX - 1) / kBX;
    const int64_t tiles = xblocks * ((g.ny * g.nz + kBY - 1) / kBY);
    const int blocks = (int)(tiles < kMaxResidualBlocks ? tiles : kMaxResidualBlocks);
    hipLaunchKernelGGL((k_residual<S, DIM, ST>), dim3(blocks), dim3(kBX, kBY), 0, s,
                       (const S*)u, (const S*)b, (S*)r, g, h2, xblocks, tiles, partials);
    cs_status st = check_launch("residual");
    if (st != CS_OK) return st;
    return launch_residual_finish(partials, blocks, norms, s);
}

}  // namespace

#define CS_DISPATCH(FN, dtype, dim, stencil, ...)                                         \
    do {                                                                                  \
        if (dtype == 0) {                                                                 \
            if (dim == 2) return stencil == FD ? FN<double, 2, FD>(__VA_ARGS__)           \
                                               : FN<double, 2, Q1>(__VA_ARGS__);          \
            return stencil == FD ? FN<double, 3, FD>(__VA_ARGS__)                         \
                                 : FN<double, 3, Q1>(__VA_ARGS__);                        \
        }                                                                                 \
        if (dim == 2) return stencil == FD ? FN<float, 2, FD>(__VA_ARGS__)                \
                                           : FN<float, 2, Q1>(__VA_ARGS__);               \
        return stencil == FD ? FN<float, 3, FD>(__VA_ARGS__) : FN<float, 3, Q1>(__VA_ARGS__); \
    } while (0)

template <int DIM, int ST>
cs_status ir_residual_t(const Geo& g, const void* x, const void* b, double h2, double inv_scale,
                        const Geo& g2, void* r32, void* e32, Partial* partials, double* norms,
                        hipStream_t s)
{
    const int64_t xblocks = (g.nx + kBX - 1) / kBX;
    const int64_t tiles = xblocks * ((g.ny * g.nz + kBY - 1) / kBY);
    const int blocks = (int)(tiles < kMaxResidualBlocks ? tiles : kMaxResidualBlocks);
    hipLaunchKernelGGL((k_ir_residual<DIM, ST>), dim3(blocks), dim3(kBX, kBY), 0, s,
                       (const double*)x, (const double*)b, g, h2, inv_scale, g2, (float*)r32,
                       (float*)e32, xblocks, tiles, partials);
    cs_status st = check_launch("ir residual");
    if (st != CS_OK) return st;
    return launch_residual_finish(partials, blocks, norms, s);
}

cs_status launch_ir_residual(int dim, int stencil, const Geo& g, const void* x, const void* b,
                             double h2, double inv_scale, const Geo& g2, void* r32, void* e32,
                             Partial* partials, double* norms, hipStream_t s)
{
    if (dim == 3 && residual3_stream_fits(g) && stream_supported(g2))
        return launch_ir_residual3(stencil, g, x, b, h2, inv_scale, g2, r32, e32, partials, norms, s);
    if (dim == 2)
        return stencil == FD ? ir_residual_t<2, FD>(g, x, b, h2, inv_scale, g2, r32, e32, partials, norms, s)
                             : ir_residual_t<2, Q1>(g, x, b, h2, inv_scale, g2, r32, e32, partials, norms, s);
    return stencil == FD ? ir_residual_t<3, FD>(g, x, b, h2, inv_scale, g2, r32, e32, partials, norms, s)
                         : ir_residual_t<3, Q1>(g, x, b, h2, inv_scale, g2, r32, e32, partials, norms, s);
}

cs_status launch_ir_update(int dim, const Geo& g, void* x, const Geo& g2, const void* e32,
                           double scale, hipStream_t s)
{
    const int64_t xblocks = (g.nx + kBX - 1) / kBX;
    const int64_t blocks = xblocks * ((g.ny * g.nz + kBY - 1) / kBY);
    if (dim == 2)
        hipLaunchKernelGGL((k_ir_update<2>), dim3((unsigned)blocks), dim3(kBX, kBY), 0, s,
                           (double*)x, g, (const float*)e32, g2, scale, xblocks);
    else
        hipLaunchKernelGGL((k_ir_update<3>), dim3((unsigned)blocks), dim3(kBX, kBY), 0, s,
                           (double*)x, g, (const float*)e32, g2, scale, xblocks);
    return check_launch("ir update");
}

cs_status launch_residual_finish(const Partial* partials, int count, double* norms, hipStream_t s)
{
    if (!norms) return CS_OK;  // the residual array alone was asked for
    hipLaunchKernelGGL(k_residual_finish, dim3(1), dim3(256), 0, s, partials, count, norms);
    return check_launch("residual finish");
}

cs_status launch_colour_pass(int dtype, int dim, int stencil, const Geo& g, void* u,
                             const void* b, double h2, int colour, hipStream_t s,
                             const StencilCost* cost)
{
    CS_DISPATCH(colour_pass_t, dtype, dim, stencil, g, u, b, h2, colour, cost, s);
}

template <typename T, int DIM, int ST>
cs_status apply_t(const Geo& g, const void* u, void* y, double h2, int cellwise, hipStream_t s)
{
    if (!cellwise) {
        const int64_t xblocks = (g.nx + kBX - 1) / kBX;
        const int64_t blocks = xblocks * ((g.ny * g.nz + kBY - 1) / kBY);
        if (blocks > 0x7fffffff) { set_error("apply: grid too large"); return CS_EUNSUPPORTED; }
        hipLaunchKernelGGL((k_apply<T, DIM, ST>), dim3((unsigned)blocks), dim3(kBX, kBY), 0, s,
                           (const T*)u, (T*)y, g, (T)h2, xblocks);
        return check_launch("apply (stencil form)");
    }
    const int64_t all = (g.nx + 2) * (g.ny + 2) * (DIM == 3 ? g.nz + 2 : 1);
    const int64_t fblocks = (all + 255) / 256;
    if (fblocks > 0x7fffffff) { set_error("apply: grid too large"); return CS_EUNSUPPORTED; }
    hipLaunchKernelGGL((k_fill_or_scale<T, DIM>), dim3((unsigned)fblocks), dim3(256), 0, s, (T*)y, g,
                       (T)h2, 0);
    for (int c = 0; c < (1 << DIM); ++c) {
        // lower corners i = bx, bx + 2, ... <= nx (the cell's far vertex i + 1 <= nx + 1)
        const int64_t cx = (g.nx - (c & 1)) / 2 + 1;
        const int64_t cy = (g.ny - ((c >> 1) & 1)) / 2 + 1;
        const int64_t cz = DIM == 3 ? (g.nz - ((c >> 2) & 1)) / 2 + 1 : 1;
        const int64_t blocks = (cx * cy * cz + 255) / 256;
        hipLaunchKernelGGL((k_cell_pass<T, DIM>), dim3((unsigned)blocks), dim3(256), 0, s,
                           (const T*)u, (T*)y, g, c, cx, cy, cz);
    }
    hipLaunchKernelGGL((k_fill_or_scale<T, DIM>), dim3((unsigned)fblocks), dim3(256), 0, s, (T*)y, g,
                       (T)h2, 1);
    return check_launch("apply (cell-wise)");
}

cs_status launch_lex_sweep(int dtype, int dim, int stencil, const Geo& g, void* u, const void* b,
                           double h2, hipStream_t s)
{
    CS_DISPATCH(lex_sweep_t, dtype, dim, stencil, g, u, b, h2, s);
}

cs_status launch_fill_uniform(int dtype, int dim, const Geo& g, void* a, uint64_t seed, hipStream_t s)
{
    const int64_t n = g.nx * g.ny * g.nz;
    const int64_t blocks = (n + 255) / 256;
    if (blocks > 0x7fffffff) { set_error("fill: grid too large"); return CS_EUNSUPPORTED; }
    if (dtype == 0) {
        if (dim == 2) hipLaunchKernelGGL((k_fill_uniform<double, 2>), dim3((unsigned)blocks), dim3(256), 0, s, (double*)a, g, seed);
        else hipLaunchKernelGGL((k_fill_uniform<double, 3>), dim3((unsigned)blocks), dim3(256), 0, s, (double*)a, g, seed);
    } else {
        if (dim == 2) hipLaunchKernelGGL((k_fill_uniform<float, 2>), dim3((unsigned)blocks), dim3(256), 0, s, (float*)a, g, seed);
        else hipLaunchKernelGGL((k_fill_uniform<float, 3>), dim3((unsigned)blocks), dim3(256), 0, s, (float*)a, g, seed);
    }
    return check_launch("seeded fill");
}

cs_status launch_apply(int dtype, int dim, int stencil, const Geo& g, const void* u, void* y,
                       double h2, int cellwise, hipStream_t s)
{
    CS_DISPATCH(apply_t, dtype, dim, stencil, g, u, y, h2, cellwise, s);
}

cs_status launch_jacobi(int dtype, int dim, int stencil, const Geo& g, const void* src,
                        void* dst, const void* b, double h2, double omega, hipStream_t s)
{
    if (dim == 3 && stream_supported(g))
        return launch_jacobi3_stream(dtype, stencil, g, src, dst, b, h2, omega, s);
    CS_DISPATCH(jacobi_t, dtype, dim, stencil, g, src, dst, b, h2, omega, s);
}

cs_status launch_residual(int dtype, int dim, int stencil, const Geo& g, const void* u,
                          const void* b, void* r, double h2, Partial* partials,
                          double* norms, hipStream_t s)
{
    if (dim == 3 && residual3_stream_fits(g))
        return launch_residual3_stream(dtype, stencil, g, u, b, r, h2, partials, norms, s);
    CS_DISPATCH(residual_t, dtype, dim, stencil, g, u, b, r, h2, partials, norms, s);
}

cs_status launch_halo_copy(int dtype, int dim, const Geo& g, const void* src, void* dst,
                           hipStream_t s)
{
    const int64_t wx = g.nx + 2;
    const int64_t per = 2 * wx + 2 * g.ny;
    const int64_t total = dim == 3 ? 2 * wx * (g.ny + 2) + g.nz * per : per;
    const int64_t blocks = (total + 255) / 256;
    if (dtype == 0) {
        if (dim == 2)
            hipLaunchKernelGGL((k_halo_copy<double, 2>), dim3((unsigned)blocks), dim3(256), 0, s,
                               (const double*)src, (double*)dst, g, total);
        else
            hipLaunchKernelGGL((k_halo_copy<double, 3>), dim3((unsigned)blocks), dim3(256), 0, s,
                               (const double*)src, (double*)dst, g, total);
    } else {
        if (dim == 2)
            hipLaunchKernelGGL((k_halo_copy<float, 2>), dim3((unsigned)blocks), dim3(256), 0, s,
                               (const float*)src, (float*)dst, g, total);
        else
            hipLaunchKernelGGL((k_halo_copy<float, 3>), dim3((unsigned)blocks), dim3(256), 0, s,
                               (const float*)src, (float*)dst, g, total);
    }
    return check_launch("halo copy");
}

cs_status launch_interior_copy(int dtype, int dim, const Geo& g, const void* src, void* dst,
                               hipStream_t s)
{
    const int64_t xblocks = (g.nx + kBX - 1) / kBX;
    const int64_t blocks = xblocks * ((g.ny * g.nz + kBY - 1) / kBY);
    if (dtype == 0) {
        if (dim == 2)
            hipLaunchKernelGGL((k_interior_copy<double, 2>), dim3((unsigned)blocks), dim3(kBX, kBY),
                               0, s, (const double*)src, (double*)dst, g, xblocks);
        else
            hipLaunchKernelGGL((k_interior_copy<double, 3>), dim3((unsigned)blocks), dim3(kBX, kBY),
                               0, s, (const double*)src, (double*)dst, g, xblocks);
    } else {
        if (dim == 2)
            hipLaunchKernelGGL((k_interior_copy<float, 2>), dim3((unsigned)blocks), dim3(kBX, kBY),
                               0, s, (const float*)src, (float*)dst, g, xblocks);
        else
            hipLaunchKernelGGL((k_interior_copy<float, 3>), dim3((unsigned)blocks), dim3(kBX, kBY),
                               0, s, (const float*)src, (float*)dst, g, xblocks);
    }
    return check_launch("interior copy");
}

}  // namespace cs
