// Persistent colour sweeps with a device-wide barrier between colours: the
// Hyb-sync form of the colouring (Sec. 5, Algorithm 1), one parallel region
// for all sweeps with a barrier after each colour, instead of a fork and join
// (a launch) per colour.
//
// One cooperative launch holds every workgroup resident.  For each sweep and
// colour, the workgroups update that colour's points in a grid-stride loop --
// the same point update, in place, as the one-launch-per-colour pass, so the
// iterate is the same bit for bit -- and then meet at a device-wide barrier.
// Every workgroup runs the same number of barriers, so all of them reach the
// end of the kernel.
#include "cs_device.h"
#include "cs_internal.h"

#include <stdint.h>

namespace cs {

namespace {

// polls (each followed by a short sleep) before a barrier gives up waiting
constexpr unsigned kSpinLimit = 1u << 24;

// Device-wide barrier.  bar[0] counts arrivals, bar[1] is the generation,
// bar[2] counts waits that gave up.  The last workgroup to arrive resets the
// count and starts the next generation; the others poll the generation.  A
// workgroup that polls kSpinLimit times without seeing it records a failure
// and goes on, so a barrier cannot wait forever (the result is then not to be
// trusted, and cs_gs_sync_failures reports it).  The workgroup barrier
// completes every wave's stores into the XCD's L2; one device-scope fence by
// the first thread then writes them back before it arrives, and one after the
// wait invalidates the L2 and the CU's L1, so the next colour reads the values
// the other workgroups, on any XCD, wrote.  (A fence in every wave costs a
// write-back and invalidation of the L2 per wave: ~30 us per barrier.)
__device__ void grid_barrier(unsigned* bar, unsigned nblocks)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned gen = __hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned arrived =
            __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (arrived == nblocks - 1) {
            __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(&bar[1], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            unsigned spins = 0;
            while (__hip_atomic_load(&bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                if (++spins == kSpinLimit) {
                    __hip_atomic_fetch_add(&bar[2], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        __threadfence();
    }
    __syncthreads();
}

// Number of points of colour c and the point of index w among them.
struct ColourSet {
    int64_t i0, j0, k0;  // first point (Q1) or row start data (FD)
    int64_t cx, cy, cz;  // counts along x, y, z (FD: cx = slots per row)
    int64_t total;
};

template <int DIM, int ST>
__device__ inline ColourSet colour_set(const Geo& g, int c)
{
    ColourSet s;
    if (ST == FD) {
        s.i0 = s.j0 = s.k0 = 0;
        s.cx = (g.nx + 1) / 2;  // slots per row; the row's first x depends on the row
        s.cy = g.ny;
        s.cz = DIM == 3 ? g.nz : 1;
    } else {
        const int px = c & 1, py = (c >> 1) & 1, pz = (c >> 2) & 1;
        s.i0 = 1 + ((px + g.parity) & 1);
        s.j0 = 1 + ((py + g.parity) & 1);
        s.k0 = DIM == 3 ? 1 + ((pz + g.parity) & 1) : 1;
        s.cx = s.i0 <= g.nx ? (g.nx - s.i0) / 2 + 1 : 0;
        s.cy = s.j0 <= g.ny ? (g.ny - s.j0) / 2 + 1 : 0;
        s.cz = DIM == 3 ? (s.k0 <= g.nz ? (g.nz - s.k0) / 2 + 1 : 0) : 1;
    }
    s.total = s.cx * s.cy * s.cz;
    return s;
}

constexpr int kSyncThreads = 1024;

// The points of colour c taken by thread tid of nthreads, each set to its
// colour-pass value in place (the same update as the one-launch-per-colour
// pass).
template <typename T, int DIM, int ST>
__device__ __forceinline__ void colour_points(T* u, const T* __restrict__ b, const Geo& g, T h2,
                                              int c, int64_t tid, int64_t nthreads)
{
    const int64_t sy = g.sy, sz = g.sz;
    const ColourSet cs = colour_set<DIM, ST>(g, c);
    for (int64_t w = tid; w < cs.total; w += nthreads) {
        const int64_t m = w % cs.cx, n = (w / cs.cx) % cs.cy, l = w / (cs.cx * cs.cy);
        int64_t i, j, k;
        if (ST == FD) {
            j = 1 + n;
            k = 1 + l;
            const int64_t kk = DIM == 3 ? k - 1 : 0;
            i = 1 + ((c + (j - 1) + kk + g.parity) & 1) + 2 * m;
            if (i > g.nx) continue;
        } else {
            i = cs.i0 + 2 * m;
            j = cs.j0 + 2 * n;
            k = cs.k0 + 2 * l;
        }
        const int64_t q = (DIM == 3 ? k * sz : 0) + j * sy + i;
        auto ld = [&](int ox, int oy, int oz) { return u[q + oz * sz + oy * sy + ox]; };
        u[q] = gs_value<T, DIM, ST>(h2, b[q], ld);
    }
}

template <typename T, int DIM, int ST>
__global__ void __launch_bounds__(kSyncThreads)
k_sync_sweeps(T* u, const T* __restrict__ b, Geo g, T h2, int nsweeps, unsigned* bar)
{
    constexpr int NC = num_colours<ST, DIM>();
    const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int sw = 0; sw < nsweeps; ++sw) {
        for (int c = 0; c < NC; ++c) {
            colour_points<T, DIM, ST>(u, b, g, h2, c, tid, nthreads);
            grid_barrier(bar, gridDim.x);
        }
    }
}

// All sweeps of a small grid in one workgroup: the colours in order, a
// workgroup barrier after each (the workgroup's global stores are visible to
// its own threads after the barrier).  One launch instead of one per colour.
constexpr int kBlockThreads = 1024;

template <typename T, int DIM, int ST>
__global__ void __launch_bounds__(kBlockThreads)
k_block_sweeps(T* u, const T* __restrict__ b, Geo g, T h2, int nsweeps)
{
    constexpr int NC = num_colours<ST, DIM>();
    for (int sw = 0; sw < nsweeps; ++sw)
        for (int c = 0; c < NC; ++c) {
            colour_points<T, DIM, ST>(u, b, g, h2, c, threadIdx.x, blockDim.x);
            __syncthreads();
        }
}

template <typename T, int DIM, int ST>
cs_status block_sweeps_t(const Geo& g, void* u, const void* b, double h2, int nsweeps,
                         hipStream_t s)
{
    // threads: about one per point of the largest colour, whole wavefronts
    const int64_t pts = g.nx * g.ny * (DIM == 3 ? g.nz : 1);
    int64_t nt = (pts / 2 + 63) / 64 * 64;
    if (nt > kBlockThreads) nt = kBlockThreads;
    if (nt < 64) nt = 64;
    hipLaunchKernelGGL((k_block_sweeps<T, DIM, ST>), dim3(1), dim3((unsigned)nt), 0, s, (T*)u,
                       (const T*)b, g, (T)h2, nsweeps);
    return check_launch("one-workgroup sweeps");
}

// ---------------------------------------------------------------------------
// The Hyb-depend form (Sec. 5): no barrier at all between colours.  The grid
// is cut into boxes ("tiles"); a tile may run colour phase p (sweep p / c,
// colour p % c) once every neighbouring tile has finished phase p - 1, and it
// publishes the number of phases it has finished in a counter of its own.  A
// tile is then never more than one phase ahead of a neighbour, so every point
// update reads exactly the values the colour passes give it (colours before
// its own from this sweep, after it from the last), and the iterate is the
// colour passes' bit for bit.  Workgroups take tiles t = blockIdx, blockIdx +
// grid, ... for every phase in turn; a cooperative launch keeps all of them
// resident, so a waited-for tile always progresses (by induction on the
// phase).  Publishing and observing follow the device-wide barrier above: a
// workgroup barrier, one device-scope fence by the first thread, a release
// store (or acquire loads, one lane per neighbour, then the fence).  Each wait
// is bounded; a wait that gives up counts a failure and raises an abort flag
// that ends every other wait at once, so the kernel always finishes.
constexpr int kDepTX3 = 32, kDepTY3 = 16, kDepTZ3 = 8;
constexpr int kDepTX2 = 64, kDepTY2 = 32;
constexpr int kDepThreads = 512;

template <int DIM, int ST>
__device__ inline int colour_of(int64_t i, int64_t j, int64_t k, int parity)
{
    if (ST == FD) return (int)(((i - 1) + (j - 1) + (DIM == 3 ? k - 1 : 0) + parity) & 1);
    const int px = (int)((i - 1 + parity) & 1), py = (int)((j - 1 + parity) & 1);
    const int pz = DIM == 3 ? (int)((k - 1 + parity) & 1) : 0;
    return px + 2 * py + 4 * pz;
}

// Clears the barrier's arrival count before a persistent launch: a barrier
// whose wait gave up leaves the count out of step with the generation, and the
// next launch must not inherit that.  The generation word may start anywhere.
__global__ void k_barrier_reset(unsigned* bar)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) bar[0] = 0u;
}

__global__ void k_dep_reset(unsigned* bar, int64_t ntiles)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) bar[3] = 0u;
    if (i < ntiles) bar[4 + i] = 0u;
}

template <typename T, int DIM, int ST>
__global__ void __launch_bounds__(kDepThreads)
k_dep_sweeps(T* u, const T* __restrict__ b, Geo g, T h2, int nsweeps, int64_t tnx, int64_t tny,
             int64_t tnz, int tzd, unsigned* bar)
{
    constexpr int NC = num_colours<ST, DIM>();
    constexpr int TX = DIM == 3 ? kDepTX3 : kDepTX2, TY = DIM == 3 ? kDepTY3 : kDepTY2;
    const int TZ = DIM == 3 ? tzd : 1;  // planes per tile
    constexpr int NB = DIM == 3 ? 27 : 9;  // the tile and its neighbours
    unsigned* done = bar + 4;
    const int64_t ntiles = tnx * tny * tnz;
    const int64_t sy = g.sy, sz = g.sz;
    const int phases = nsweeps * NC;
    for (int p = 0; p < phases; ++p) {
        const int c = p % NC;
        for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
            const int64_t tx = t % tnx, ty = (t / tnx) % tny, tz = t / (tnx * tny);
            if (p > 0 && (int)threadIdx.x < NB) {
                const int o = threadIdx.x;
                const int64_t nx = tx + o % 3 - 1, ny = ty + (o / 3) % 3 - 1;
                const int64_t nz = DIM == 3 ? tz + o / 9 - 1 : tz;
                const bool self = nx == tx && ny == ty && nz == tz;
                if (!self && nx >= 0 && nx < tnx && ny >= 0 && ny < tny && nz >= 0 && nz < tnz) {
                    const unsigned* w = &done[(nz * tny + ny) * tnx + nx];
                    unsigned spins = 0;
                    while (__hip_atomic_load(w, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < (unsigned)p) {
                        if (__hip_atomic_load(&bar[3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
                        if (++spins == kSpinLimit) {
                            __hip_atomic_fetch_add(&bar[2], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            __hip_atomic_store(&bar[3], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            break;
                        }
                        __builtin_amdgcn_s_sleep(2);
                    }
                }
            }
            __syncthreads();
            if (threadIdx.x == 0) __threadfence();
            __syncthreads();
            const int64_t x0 = 1 + tx * TX, y0 = 1 + ty * TY, z0 = 1 + tz * TZ;
            const int tile_pts = TX * TY * TZ;
            for (int w = threadIdx.x; w < tile_pts; w += blockDim.x) {
                const int64_t i = x0 + w % TX, j = y0 + (w / TX) % TY;
                const int64_t k = DIM == 3 ? z0 + w / (TX * TY) : 1;
                if (i > g.nx || j > g.ny || (DIM == 3 && k > g.nz)) continue;
                if (colour_of<DIM, ST>(i, j, k, g.parity) != c) continue;
                const int64_t q = (DIM == 3 ? k * sz : 0) + j * sy + i;
                auto ld = [&](int ox, int oy, int oz) { return u[q + oz * sz + oy * sy + ox]; };
                u[q] = gs_value<T, DIM, ST>(h2, b[q], ld);
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                __threadfence();
                __hip_atomic_store(&done[t], (unsigned)(p + 1), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
}

template <typename T, int DIM, int ST>
cs_status dep_sweeps_t(const Geo& g, void* u, const void* b, double h2, int nsweeps, unsigned* bar,
                       hipStream_t s)
{
    auto kern = k_dep_sweeps<T, DIM, ST>;
    static const int64_t resident = [&] {
        int per_cu = 0, dev = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kDepThreads, 0) != hipSuccess ||
            hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
            (void)hipGetLastError();
            return (int64_t)0;
        }
        // one workgroup per CU: fewer fences per phase
        return (int64_t)(per_cu > 0 ? 1 : 0) * cus;
    }();
    if (resident <= 0) {
        set_error("dependency sweep: no resident workgroups");
        return CS_EHIP;
    }
    // tiles of kDepTZ3 planes (the counters are sized for these), deepened in z
    // to about one tile per resident workgroup: one publication per workgroup
    // and phase where the grid allows
    int64_t tnx, tny, tnz;
    dep_tile_counts(g, DIM, &tnx, &tny, &tnz);
    int tzd = kDepTZ3;
    if (DIM == 3) {
        const int64_t f = (tnx * tny * tnz + resident - 1) / resident;
        tzd = (int)(kDepTZ3 * (f < 1 ? 1 : f));
        if (tzd > g.nz) tzd = (int)g.nz;
        if (tzd < 1) tzd = 1;
        tnz = (g.nz + tzd - 1) / tzd;
    }
    const int64_t ntiles = tnx * tny * tnz;
    hipLaunchKernelGGL(k_dep_reset, dim3((unsigned)((ntiles + 255) / 256)), dim3(256), 0, s, bar, ntiles);
    cs_status st = check_launch("dependency counters reset");
    if (st != CS_OK) return st;
    const int64_t blocks = ntiles < resident ? ntiles : resident;
    Geo gg = g;
    T h2t = (T)h2;
    int ns = nsweeps;
    void* args[] = {&u, (void*)&b, &gg, &h2t, &ns, &tnx, &tny, &tnz, &tzd, &bar};
    hipError_t e = hipLaunchCooperativeKernel((const void*)kern, dim3((unsigned)blocks),
                                              dim3(kDepThreads), args, 0, s);
    if (e != hipSuccess) return hip_fail(e, "hipLaunchCooperativeKernel");
    return check_launch("dependency-driven colour sweeps");
}

template <typename T, int DIM, int ST>
cs_status sync_sweeps_t(const Geo& g, void* u, const void* b, double h2, int nsweeps,
                        unsigned* bar, hipStream_t s)
{
    auto kern = k_sync_sweeps<T, DIM, ST>;
    static const int64_t resident = [&] {
        int per_cu = 0, dev = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kSyncThreads, 0) != hipSuccess ||
            hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
            (void)hipGetLastError();
            return (int64_t)0;
        }
        // one workgroup per CU: fewer workgroups, fewer fences per barrier
        return (int64_t)(per_cu > 0 ? 1 : 0) * cus;
    }();
    if (resident <= 0) {
        set_error("persistent sweep: no resident workgroups");
        return CS_EHIP;
    }
    // enough workgroups for the largest colour, at most what fits at once
    const int64_t pts = g.nx * g.ny * (DIM == 3 ? g.nz : 1);
    int64_t blocks = (pts / 2 + kSyncThreads - 1) / kSyncThreads;
    if (blocks > resident) blocks = resident;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_barrier_reset, dim3(1), dim3(64), 0, s, bar);
    cs_status st = check_launch("barrier reset");
    if (st != CS_OK) return st;
    Geo gg = g;
    T h2t = (T)h2;
    int ns = nsweeps;
    void* args[] = {&u, (void*)&b, &gg, &h2t, &ns, &bar};
    hipError_t e = hipLaunchCooperativeKernel((const void*)kern, dim3((unsigned)blocks),
                                              dim3(kSyncThreads), args, 0, s);
    if (e != hipSuccess) return hip_fail(e, "hipLaunchCooperativeKernel");
    return check_launch("persistent colour sweeps");
}

}  // namespace

void dep_tile_counts(const Geo& g, int dim, int64_t* tnx, int64_t* tny, int64_t* tnz)
{
    const int64_t TX = dim == 3 ? kDepTX3 : kDepTX2, TY = dim == 3 ? kDepTY3 : kDepTY2;
    const int64_t TZ = dim == 3 ? kDepTZ3 : 1;
    *tnx = (g.nx + TX - 1) / TX;
    *tny = (g.ny + TY - 1) / TY;
    *tnz = dim == 3 ? (g.nz + TZ - 1) / TZ : 1;
}

cs_status launch_dep_sweeps(int dtype, int dim, int stencil, const Geo& g, void* u, const void* b,
                            double h2, int nsweeps, unsigned* bar, hipStream_t s)
{
    if (dtype == 0) {
        if (dim == 2)
            return stencil == FD ? dep_sweeps_t<double, 2, FD>(g, u, b, h2, nsweeps, bar, s)
                                 : dep_sweeps_t<double, 2, Q1>(g, u, b, h2, nsweeps, bar, s);
        return stencil == FD ? dep_sweeps_t<double, 3, FD>(g, u, b, h2, nsweeps, bar, s)
                             : dep_sweeps_t<double, 3, Q1>(g, u, b, h2, nsweeps, bar, s);
    }
    if (dim == 2)
        return stencil == FD ? dep_sweeps_t<float, 2, FD>(g, u, b, h2, nsweeps, bar, s)
                             : dep_sweeps_t<float, 2, Q1>(g, u, b, h2, nsweeps, bar, s);
    return stencil == FD ? dep_sweeps_t<float, 3, FD>(g, u, b, h2, nsweeps, bar, s)
                         : dep_sweeps_t<float, 3, Q1>(g, u, b, h2, nsweeps, bar, s);
}

cs_status launch_block_sweeps(int dtype, int dim, int stencil, const Geo& g, void* u,
                              const void* b, double h2, int nsweeps, hipStream_t s)
{
    if (dtype == 0) {
        if (dim == 2)
            return stencil == FD ? block_sweeps_t<double, 2, FD>(g, u, b, h2, nsweeps, s)
                                 : block_sweeps_t<double, 2, Q1>(g, u, b, h2, nsweeps, s);
        return stencil == FD ? block_sweeps_t<double, 3, FD>(g, u, b, h2, nsweeps, s)
                             : block_sweeps_t<double, 3, Q1>(g, u, b, h2, nsweeps, s);
    }
    if (dim == 2)
        return stencil == FD ? block_sweeps_t<float, 2, FD>(g, u, b, h2, nsweeps, s)
                             : block_sweeps_t<float, 2, Q1>(g, u, b, h2, nsweeps, s);
    return stencil == FD ? block_sweeps_t<float, 3, FD>(g, u, b, h2, nsweeps, s)
                         : block_sweeps_t<float, 3, Q1>(g, u, b, h2, nsweeps, s);
}

cs_status launch_sync_sweeps(int dtype, int dim, int stencil, const Geo& g, void* u,
                             const void* b, double h2, int nsweeps, unsigned* bar, hipStream_t s)
{
    if (dtype == 0) {
        if (dim == 2)
            return stencil == FD ? sync_sweeps_t<double, 2, FD>(g, u, b, h2, nsweeps, bar, s)
                                 : sync_sweeps_t<double, 2, Q1>(g, u, b, h2, nsweeps, bar, s);
        return stencil == FD ? sync_sweeps_t<double, 3, FD>(g, u, b, h2, nsweeps, bar, s)
                             : sync_sweeps_t<double, 3, Q1>(g, u, b, h2, nsweeps, bar, s);
    }
    if (dim == 2)
        return stencil == FD ? sync_sweeps_t<float, 2, FD>(g, u, b, h2, nsweeps, bar, s)
                             : sync_sweeps_t<float, 2, Q1>(g, u, b, h2, nsweeps, bar, s);
    return stencil == FD ? sync_sweeps_t<float, 3, FD>(g, u, b, h2, nsweeps, bar, s)
                         : sync_sweeps_t<float, 3, Q1>(g, u, b, h2, nsweeps, bar, s);
}

}  // namespace cs
