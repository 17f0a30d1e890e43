// Fused Gauss-Seidel sweeps of 2D grids: S whole sweeps per launch on a tile
// held in LDS (the colouring of Sec. 3, red-black for the 5-point and four
// parity colours for the 9-point stencil, colours in canonical order).
//
// A tile of TX x TY interior points loads the previous iterate u on the
// region grown by H = S * c points (c colours) and b on the same region, runs
// the S * c colour phases in order -- phase p updates the points of its colour
// on the region grown by H - 1 - p, in place in LDS, since each phase needs
// its neighbours' values from the phase before it one point further out --
// and writes the tile to dst.  Within a phase a point reads only points of
// other colours (both stencils couple no two points of one colour), so the
// in-place updates do not race, and every value equals that of the S sweeps
// of colour passes bit for bit (same ordered neighbour sum).  Tiles read the
// previous iterate around them, so the result goes to the other array.
//
// A 256 x 256 grid is latency-bound (a FP64 array is 0.5 MB), and S sweeps
// per launch replace 2 S or 4 S launches; on large 2D grids the tile reads u
// and b once for S sweeps.
#include "cs_device.h"
#include "cs_internal.h"

#include <stdint.h>

namespace cs {

namespace {

template <int ST>
__device__ __forceinline__ int colour_2d(int64_t x, int64_t y, int parity)
{
    if (ST == FD) return (int)(((x - 1) + (y - 1) + parity) & 1);
    return (int)(((x - 1 + parity) & 1) + 2 * ((y - 1 + parity) & 1));
}

template <typename T, int ST, int TX, int TY, int S, int NT>
__global__ void __launch_bounds__(NT)
k_fused2d(const T* __restrict__ src, T* __restrict__ dst, const T* __restrict__ b, Geo g, T h2,
          int tiles_x)
{
    constexpr int NC = ST == FD ? 2 : 4;
    constexpr int H = S * NC;
    constexpr int W = TX + 2 * H, HH = TY + 2 * H, N = W * HH;
    constexpr int M = (N + NT - 1) / NT;  // loaded points per thread
    constexpr int MP = ((TX + 2 * H - 2) * (TY + 2 * H - 2) + NT - 1) / NT;  // phase points
    __shared__ T lu[N];
    __shared__ T lb[N];
    const int tid = threadIdx.x;
    const int64_t tile = blockIdx.x;
    const int64_t x0 = 1 + (tile % tiles_x) * TX, y0 = 1 + (tile / tiles_x) * TY;
    const int64_t ox0 = x0 - H, oy0 = y0 - H;  // region origin

    // every load in flight before the first LDS store
    {
        T ru[M], rb[M];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int c = tid + NT * m;
            const int64_t x = ox0 + c % W, y = oy0 + c / W;
            const bool dom = c < N && x >= 0 && x <= g.nx + 1 && y >= 0 && y <= g.ny + 1;
            const bool inner = dom && x >= 1 && x <= g.nx && y >= 1 && y <= g.ny;
            ru[m] = dom ? src[y * g.sy + x] : T(0);
            rb[m] = inner ? b[y * g.sy + x] : T(0);
        }
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int c = tid + NT * m;
            if (c < N) {
                lu[c] = ru[m];
                lb[c] = rb[m];
            }
        }
    }
    __syncthreads();

    // Phase p updates its colour on the tile grown by H - 1 - p.  A thread
    // computes all its points of the phase before storing any (points of one
    // colour never read each other), so the LDS loads of its points overlap.
#pragma unroll
    for (int p = 0; p < S * NC; ++p) {
        const int colour = p % NC;
        const int r = H - 1 - p;
        const int w = TX + 2 * r, npts = w * (TY + 2 * r);
        int cidx[MP];
        T val[MP];
#pragma unroll
        for (int i = 0; i < MP; ++i) {
            const int t = tid + NT * i;
            const int lx = H - r + t % w, ly = H - r + t / w;
            const int64_t x = ox0 + lx, y = oy0 + ly;
            const bool upd = t < npts && x >= 1 && x <= g.nx && y >= 1 && y <= g.ny &&
                             colour_2d<ST>(x, y, g.parity) == colour;
            const int c = ly * W + lx;
            cidx[i] = upd ? c : -1;
            if (upd) {
                auto ld = [&](int ox, int oy, int oz) -> T { return lu[c + oy * W + ox]; };
                val[i] = gs_value<T, 2, ST>(h2, lb[c], ld);
            }
        }
#pragma unroll
        for (int i = 0; i < MP; ++i)
            if (cidx[i] >= 0) lu[cidx[i]] = val[i];
        __syncthreads();
    }

    for (int t = tid; t < TX * TY; t += NT) {
        const int64_t x = x0 + t % TX, y = y0 + t / TX;
        if (x <= g.nx && y <= g.ny) st_stream(dst + y * g.sy + x, lu[(t / TX + H) * W + t % TX + H]);
    }
}

// S weighted Jacobi sweeps of a 2D grid per launch: the same LDS-resident
// tile with a halo of H = S points (one per sweep) and two LDS buffers; sweep
// s computes the region grown by H - 1 - s from the buffer the sweep before
// wrote, with the same expression as the one-sweep kernel, so the values
// equal S separate sweeps bit for bit.  Boundary points hold their Dirichlet
// values in both buffers.
template <typename T, int ST, int TX, int TY, int S, int NT>
__global__ void __launch_bounds__(NT)
k_jacobi2d(const T* __restrict__ src, T* __restrict__ dst, const T* __restrict__ b, Geo g, T h2,
           T omega, int tiles_x)
{
    constexpr int H = S;
    constexpr int W = TX + 2 * H, HH = TY + 2 * H, N = W * HH;
    constexpr int M = (N + NT - 1) / NT;
    constexpr int MP = ((TX + 2 * H - 2) * (TY + 2 * H - 2) + NT - 1) / NT;
    __shared__ T lu[2][N];
    __shared__ T lb[N];
    const int tid = threadIdx.x;
    const int64_t tile = blockIdx.x;
    const int64_t x0 = 1 + (tile % tiles_x) * TX, y0 = 1 + (tile / tiles_x) * TY;
    const int64_t ox0 = x0 - H, oy0 = y0 - H;

    {
        T ru[M], rb[M];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int c = tid + NT * m;
            const int64_t x = ox0 + c % W, y = oy0 + c / W;
            const bool dom = c < N && x >= 0 && x <= g.nx + 1 && y >= 0 && y <= g.ny + 1;
            const bool inner = dom && x >= 1 && x <= g.nx && y >= 1 && y <= g.ny;
            ru[m] = dom ? src[y * g.sy + x] : T(0);
            rb[m] = inner ? b[y * g.sy + x] : T(0);
        }
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int c = tid + NT * m;
            if (c < N) {
                lu[0][c] = ru[m];
                lu[1][c] = ru[m];
                lb[c] = rb[m];
            }
        }
    }
    __syncthreads();

#pragma unroll
    for (int sw = 0; sw < S; ++sw) {
        const T* in = lu[sw & 1];
        T* out = lu[(sw + 1) & 1];
        const int r = H - 1 - sw;
        const int w = TX + 2 * r, npts = w * (TY + 2 * r);
#pragma unroll
        for (int i = 0; i < MP; ++i) {
            const int t = tid + NT * i;
            const int lx = H - r + t % w, ly = H - r + t / w;
            const int64_t x = ox0 + lx, y = oy0 + ly;
            if (t < npts && x >= 1 && x <= g.nx && y >= 1 && y <= g.ny) {
                const int c = ly * W + lx;
                auto ld = [&](int ox, int oy, int oz) -> T { return in[c + oy * W + ox]; };
                out[c] = jacobi_value<T, 2, ST>(h2, omega, lb[c], in[c], ld);
            }
        }
        __syncthreads();
    }

    const T* fin = lu[S & 1];
    for (int t = tid; t < TX * TY; t += NT) {
        const int64_t x = x0 + t % TX, y = y0 + t / TX;
        if (x <= g.nx && y <= g.ny) st_stream(dst + y * g.sy + x, fin[(t / TX + H) * W + t % TX + H]);
    }
}

template <typename T, int ST, int TX, int TY, int S>
cs_status jacobi2d_tile(const Geo& g, const void* src, void* dst, const void* b, double h2,
                        double omega, hipStream_t s)
{
    constexpr int NT = 1024;
    const int64_t tiles_x = (g.nx + TX - 1) / TX, tiles_y = (g.ny + TY - 1) / TY;
    const int64_t tiles = tiles_x * tiles_y;
    if (tiles > 0x7fffffff) {
        set_error("fused 2D Jacobi: too many tiles");
        return CS_EUNSUPPORTED;
    }
    hipLaunchKernelGGL((k_jacobi2d<T, ST, TX, TY, S, NT>), dim3((unsigned)tiles), dim3(NT), 0, s,
                       (const T*)src, (T*)dst, (const T*)b, g, (T)h2, (T)omega, (int)tiles_x);
    return check_launch("fused 2D Jacobi sweeps");
}

template <typename T, int ST, int TX, int TY, int S>
cs_status fused2d_tile(const Geo& g, const void* src, void* dst, const void* b, double h2,
                       hipStream_t s)
{
    constexpr int NT = 1024;
    const int64_t tiles_x = (g.nx + TX - 1) / TX, tiles_y = (g.ny + TY - 1) / TY;
    const int64_t tiles = tiles_x * tiles_y;
    if (tiles > 0x7fffffff) {
        set_error("fused 2D sweep: too many tiles");
        return CS_EUNSUPPORTED;
    }
    hipLaunchKernelGGL((k_fused2d<T, ST, TX, TY, S, NT>), dim3((unsigned)tiles), dim3(NT), 0, s,
                       (const T*)src, (T*)dst, (const T*)b, g, (T)h2, (int)tiles_x);
    return check_launch("fused 2D sweeps");
}

int device_cus()
{
    static int cus = 0;
    if (cus == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
            (void)hipGetLastError();
            cus = 256;
        }
    }
    return cus;
}

// 1024 threads per tile; 64 x 32 tiles where they still give every CU one,
// else 32 x 32 (measured: small grids are latency-bound and want more tiles,
// large ones the smaller halo share of the wider tile).
template <typename T, int ST, int S>
cs_status fused2d_t(const Geo& g, const void* src, void* dst, const void* b, double h2,
                    hipStream_t s)
{
    const int64_t wide = ((g.nx + 63) / 64) * ((g.ny + 31) / 32);
    if (wide >= device_cus()) return fused2d_tile<T, ST, 64, 32, S>(g, src, dst, b, h2, s);
    return fused2d_tile<T, ST, 32, 32, S>(g, src, dst, b, h2, s);
}

// Up to 4 red-black or 2 four-colour sweeps per launch: more sweeps need a
// wider halo, whose recomputation then costs more than the launches saved.
template <typename T, int ST>
cs_status fused2d_s(int sweeps, const Geo& g, const void* src, void* dst, const void* b, double h2,
                    hipStream_t s)
{
    switch (sweeps) {
    case 1: return fused2d_t<T, ST, 1>(g, src, dst, b, h2, s);
    case 2: return fused2d_t<T, ST, 2>(g, src, dst, b, h2, s);
    case 4:
        if (ST == FD) return fused2d_t<T, FD, 4>(g, src, dst, b, h2, s);
        break;
    default: break;
    }
    set_error("fused 2D sweep: %d sweeps per launch not available", sweeps);
    return CS_EUNSUPPORTED;
}

template <typename T, int ST, int S>
cs_status jacobi2d_t(const Geo& g, const void* src, void* dst, const void* b, double h2,
                     double omega, hipStream_t s)
{
    const int64_t wide = ((g.nx + 63) / 64) * ((g.ny + 31) / 32);
    if (wide >= device_cus()) return jacobi2d_tile<T, ST, 64, 32, S>(g, src, dst, b, h2, omega, s);
    return jacobi2d_tile<T, ST, 32, 32, S>(g, src, dst, b, h2, omega, s);
}

template <typename T, int ST>
cs_status jacobi2d_s(int sweeps, const Geo& g, const void* src, void* dst, const void* b,
                     double h2, double omega, hipStream_t s)
{
    switch (sweeps) {
    case 1: return jacobi2d_t<T, ST, 1>(g, src, dst, b, h2, omega, s);
    case 2: return jacobi2d_t<T, ST, 2>(g, src, dst, b, h2, omega, s);
    case 4: return jacobi2d_t<T, ST, 4>(g, src, dst, b, h2, omega, s);
    case 8: return jacobi2d_t<T, ST, 8>(g, src, dst, b, h2, omega, s);
    default: break;
    }
    set_error("fused 2D Jacobi: %d sweeps per launch not available", sweeps);
    return CS_EUNSUPPORTED;
}

}  // namespace

// Up to 8 Jacobi sweeps per launch on grids too small to give every CU a wide
// tile (latency-bound: fewer launches win), up to 4 on larger ones (measured:
// 256^2 56 against 46 GLUP/s, 4096^2 441 against 615).
int jacobi2d_max_sweeps(const Geo& g)
{
    const int64_t wide = ((g.nx + 63) / 64) * ((g.ny + 31) / 32);
    return wide < device_cus() ? 8 : 4;
}

cs_status launch_jacobi2d(int dtype, int stencil, int sweeps, const Geo& g, const void* src,
                          void* dst, const void* b, double h2, double omega, hipStream_t s)
{
    if (dtype == 0)
        return stencil == FD ? jacobi2d_s<double, FD>(sweeps, g, src, dst, b, h2, omega, s)
                             : jacobi2d_s<double, Q1>(sweeps, g, src, dst, b, h2, omega, s);
    return stencil == FD ? jacobi2d_s<float, FD>(sweeps, g, src, dst, b, h2, omega, s)
                         : jacobi2d_s<float, Q1>(sweeps, g, src, dst, b, h2, omega, s);
}

int fused2d_max_sweeps(int stencil)
{
    return stencil == FD ? 4 : 2;
}

cs_status launch_fused2d(int dtype, int stencil, int sweeps, const Geo& g, const void* src,
                         void* dst, const void* b, double h2, hipStream_t s)
{
    if (dtype == 0)
        return stencil == FD ? fused2d_s<double, FD>(sweeps, g, src, dst, b, h2, s)
                             : fused2d_s<double, Q1>(sweeps, g, src, dst, b, h2, s);
    return stencil == FD ? fused2d_s<float, FD>(sweeps, g, src, dst, b, h2, s)
                         : fused2d_s<float, Q1>(sweeps, g, src, dst, b, h2, s);
}

}  // namespace cs
