// Fused Gauss-Seidel sweeps: every colour of one sweep in a single pass over
// memory, reading the previous iterate from `src` and writing the new one to
// `dst` (both arrays carry the same Dirichlet halo).
//
// Red-black, 7-point (colouring of Sec. 3 with c = 2).  Red points depend only
// on black values of the previous iterate and black points only on the new red
// values, so a sweep can stream through z: at plane step k the red points of
// plane k are updated from the old black values of planes k-1..k+1, then the
// black points of plane k-1 from the new red values of planes k-2..k.  Plane
// k-1 is then final and is written out.  This is the colour order of the
// sweep, so the result equals the c in-place colour passes.
//
// Each workgroup owns an xy tile T of TX x TY interior points and a chunk of
// ZC planes.  Neighbouring tiles run independently: a tile recomputes the new
// red values on the one-point ring T+1 itself (from old values on T+2), which
// is why the two arrays are needed -- old values are never overwritten during
// the sweep.  Each thread owns columns of the region T+2 and keeps a window of
// four planes of its columns in registers (z neighbours), the in-plane
// neighbours are exchanged through two LDS planes.  Neighbour sums keep the
// lexicographic offset order of the plain sequential definition, so the
// values are bit-identical to the colour passes.
//
// Workgroups are mapped XCD by XCD: consecutive tile indices (the xy tiles of
// one z chunk) land on the same XCD so that the tiles' overlapping halo rows
// are served from that XCD's L2.
#include <cstdint>

#include "cs_tiles.h"

namespace cs {

namespace {

template <typename T, int TX, int TY, int NT, int D>
__global__ void __launch_bounds__(NT)
k_fused_fd3(const T* __restrict__ src, T* __restrict__ dst, const T* __restrict__ b, Geo g,
            T h2, FusedWork wk)
{
    const TileBox tb = tile_box<TX, TY>(g, wk.tiles_x, wk.tiles_y, wk.chunks,
                                        xcd_ordered_block(wk.nblocks));
    fd3_tile<T, TX, TY, NT, D>(src, dst, b, g, h2, tb);
}

template <typename T, int TX, int TY, int NT, int D, int NB>
__global__ void __launch_bounds__(NT)
k_fused_fd3_two(const T* __restrict__ src, T* __restrict__ dst, const T* __restrict__ b, Geo g,
                T h2, FusedWork wk)
{
    const TileBox tb = tile_box<TX, TY>(g, wk.tiles_x, wk.tiles_y, wk.chunks,
                                        xcd_ordered_block(wk.nblocks));
    fd3_tile_two<T, TX, TY, NT, D, NB>(src, dst, b, g, h2, tb);
}

template <typename T, int TX, int TY, int NT, int WPE, bool VEC>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WPE)))
k_fused_q1_3(const T* __restrict__ src, T* __restrict__ dst, const T* __restrict__ b, Geo g,
             T h2, FusedWork wk)
{
    const TileBox tb = tile_box<TX, TY>(g, wk.tiles_x, wk.tiles_y, wk.chunks,
                                        xcd_ordered_block(wk.nblocks));
    q1_3_tile_pairs<T, TX, TY, NT, true, VEC>(src, dst, b, g, h2, tb);
}

template <typename T, int TX, int TY, int NT>
__global__ void __launch_bounds__(NT)
k_fused_q1_3_two(const T* __restrict__ src, T* __restrict__ dst, const T* __restrict__ b, Geo g,
                 T h2, FusedWork wk)
{
    const TileBox tb = tile_box<TX, TY>(g, wk.tiles_x, wk.tiles_y, wk.chunks,
                                        xcd_ordered_block(wk.nblocks));
    q1_3_tile_two<T, TX, TY, NT>(src, dst, b, g, h2, tb);
}

// Resident workgroups of a kernel on the current device.  Callers keep the
// result in a static of their own template instantiation, so it is queried once
// per kernel (the library runs on devices of one kind); a cache here would be
// shared by every kernel of the same signature.
template <typename K>
int64_t resident_blocks(K kern, int nt)
{
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, nt, 0) != hipSuccess ||
        hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        return 256;
    }
    return (int64_t)(per_cu > 0 ? per_cu : 1) * cus;
}

// Chunks so that the grid is one full wave of resident workgroups, each chunk
// at least min_depth planes deep.
FusedWork plan_work(int64_t resident, const Geo& g, int tx, int ty, int min_depth = 8)
{
    FusedWork wk;
    wk.tiles_x = (int)((g.nx + tx - 1) / tx);
    wk.tiles_y = (int)((g.ny + ty - 1) / ty);
    const int64_t tiles = (int64_t)wk.tiles_x * wk.tiles_y;
    int64_t chunks = resident / tiles;
    if (chunks < 1) chunks = 1;
    if (chunks > g.nz / min_depth) chunks = g.nz / min_depth > 0 ? g.nz / min_depth : 1;
    wk.chunks = (int)chunks;
    wk.nblocks = tiles * chunks;
    return wk;
}

template <typename T, int TX, int TY, int NT, int D>
cs_status fused_fd3_t(const Geo& g, const void* src, void* dst, const void* b, double h2,
                      hipStream_t s)
{
    auto kern = k_fused_fd3<T, TX, TY, NT, D>;
    static const int64_t resident = resident_blocks(kern, NT);
    const FusedWork wk = plan_work(resident, g, TX, TY);
    hipLaunchKernelGGL(kern, dim3((unsigned)wk.nblocks), dim3(NT), 0, s, (const T*)src, (T*)dst,
                       (const T*)b, g, (T)h2, wk);
    return check_launch("fused 7-point sweep");
}

// Two sweeps per launch: the chunks carry 3 extra planes of work on each side,
// so they are kept at least 16 planes deep.
template <typename T, int TX, int TY, int NT, int D, int NB>
int64_t fused_two_resident()
{
    static const int64_t resident = resident_blocks(k_fused_fd3_two<T, TX, TY, NT, D, NB>, NT);
    return resident;
}

// Whether the double sweep's grid fills at least 3/4 of the device: with one
// workgroup per CU and chunks of 16 or more planes it leaves CUs idle on small
// grids, where two single sweeps are faster (measured: FP64 from 160^3, FP32
// from 192^3 the double sweep wins).
template <typename T, int TX, int TY, int NT, int D, int NB>
bool fused_two_fills(const Geo& g)
{
    const int64_t tiles = ((g.nx + TX - 1) / TX) * ((g.ny + TY - 1) / TY);
    return 4 * tiles * (g.nz / 16) >= 3 * fused_two_resident<T, TX, TY, NT, D, NB>();
}

template <typename T, int TX, int TY, int NT, int D, int NB>
cs_status fused_fd3_two_t(const Geo& g, const void* src, void* dst, const void* b, double h2,
                          hipStream_t s)
{
    auto kern = k_fused_fd3_two<T, TX, TY, NT, D, NB>;
    const FusedWork wk = plan_work(fused_two_resident<T, TX, TY, NT, D, NB>(), g, TX, TY, 16);
    hipLaunchKernelGGL(kern, dim3((unsigned)wk.nblocks), dim3(NT), 0, s, (const T*)src, (T*)dst,
                       (const T*)b, g, (T)h2, wk);
    return check_launch("fused 7-point double sweep");
}

// Two 27-point sweeps per launch: a chunk computes 3 extra planes of the
// first sweep on each side, so chunks are kept at least 16 planes deep.
template <typename T, int TX, int TY, int NT>
int64_t q1_two_resident()
{
    static const int64_t resident = resident_blocks(k_fused_q1_3_two<T, TX, TY, NT>, NT);
    return resident;
}

template <typename T, int TX, int TY, int NT>
cs_status fused_q1_3_two_t(const Geo& g, const void* src, void* dst, const void* b, double h2,
                           hipStream_t s)
{
    auto kern = k_fused_q1_3_two<T, TX, TY, NT>;
    const FusedWork wk = plan_work(q1_two_resident<T, TX, TY, NT>(), g, TX, TY, 16);
    hipLaunchKernelGGL(kern, dim3((unsigned)wk.nblocks), dim3(NT), 0, s, (const T*)src, (T*)dst,
                       (const T*)b, g, (T)h2, wk);
    return check_launch("fused 27-point double sweep");
}

template <typename T, int TX, int TY, int NT, int WPE>
cs_status fused_q1_3_t(const Geo& g, const void* src, void* dst, const void* b, double h2,
                       hipStream_t s, bool pairs)
{
    // two-column loads where the layout allows them; the same plan and
    // values either way
    auto kern = pairs ? k_fused_q1_3<T, TX, TY, NT, WPE, true> : k_fused_q1_3<T, TX, TY, NT, WPE, false>;
    static const int64_t resident = resident_blocks(k_fused_q1_3<T, TX, TY, NT, WPE, false>, NT);
    const FusedWork wk = plan_work(resident, g, TX, TY);
    hipLaunchKernelGGL(kern, dim3((unsigned)wk.nblocks), dim3(NT), 0, s, (const T*)src, (T*)dst,
                       (const T*)b, g, (T)h2, wk);
    return check_launch("fused 27-point sweep");
}

}  // namespace

bool fused_supported(int dtype, int dim, int stencil, const Geo& g)
{
    (void)dtype;
    (void)stencil;
    if (dim == 2) return true;  // k_fused2d.hip, 64-bit offsets
    // column offsets y*sy + x are 32-bit inside the 3D kernels
    const bool small = (g.ny + 2) * g.sy < ((int64_t)1 << 31);
    return dim == 3 && small;
}

// Tile, threads, prefetch depth and snapshot sets of the double sweep per
// precision (measured at 256^3): FP64 64 x 16 with two snapshot sets, FP32
// 64 x 32 with one.
constexpr int kF2TX = 64, kF2TY = 16, kF2NT = 1024, kF2D = 2, kF2NB = 2;
constexpr int kF2TX32 = 64, kF2TY32 = 32, kF2NT32 = 1024, kF2D32 = 2, kF2NB32 = 1;
// Tile and threads of the 27-point double sweep (one workgroup per CU: seven
// LDS planes of the region T+8).
constexpr int kQ2TX = 64, kQ2TY = 16, kQ2NT = 1024;

bool fused_two_available(int dtype, int dim, int stencil, const Geo& g)
{
    return dim == 3 && fused_supported(dtype, dim, stencil, g);
}

bool fused_two_preferred(int dtype, int dim, int stencil, const Geo& g)
{
    if (!fused_two_available(dtype, dim, stencil, g)) return false;
    if (stencil == Q1) return false;
    return dtype == 0
               ? fused_two_fills<double, kF2TX, kF2TY, kF2NT, kF2D, kF2NB>(g)
               : fused_two_fills<float, kF2TX32, kF2TY32, kF2NT32, kF2D32, kF2NB32>(g);
}

cs_status launch_fused_two(int dtype, int dim, int stencil, const Geo& g, const void* src,
                           void* dst, const void* b, double h2, hipStream_t s)
{
    if (!fused_two_available(dtype, dim, stencil, g)) {
        set_error("fused double sweep not available for this grid");
        return CS_EUNSUPPORTED;
    }
    if (stencil == Q1)
        return dtype == 0 ? fused_q1_3_two_t<double, kQ2TX, kQ2TY, kQ2NT>(g, src, dst, b, h2, s)
                          : fused_q1_3_two_t<float, kQ2TX, kQ2TY, kQ2NT>(g, src, dst, b, h2, s);
    return dtype == 0
               ? fused_fd3_two_t<double, kF2TX, kF2TY, kF2NT, kF2D, kF2NB>(
                     g, src, dst, b, h2, s)
               : fused_fd3_two_t<float, kF2TX32, kF2TY32, kF2NT32, kF2D32, kF2NB32>(
                     g, src, dst, b, h2, s);
}

bool pair_layout(const Geo& g, int dim, const void* p, size_t elem, size_t room_before, size_t room_after)
{
    return dim == 3 && ((uintptr_t)p + elem) % (2 * elem) == 0 && g.sy % 2 == 0 && g.sz % 2 == 0 &&
           g.sy >= g.nx + 3 && room_before >= elem && room_after >= elem;
}

cs_status launch_fused_sweep(int dtype, int dim, int stencil, const Geo& g, const void* src,
                             void* dst, const void* b, double h2, hipStream_t s, bool src_pairs)
{
    if (dim != 3 || !fused_supported(dtype, dim, stencil, g)) {
        set_error("fused sweep not available for this grid");
        return CS_EUNSUPPORTED;
    }
    if (stencil == Q1)
        // the pair update row by row: FP64 with 512 threads (two workgroups
        // of 8 waves per CU, 107 VGPRs), FP32 with 256 (measured at 256^3 and
        // 512^3)
        // (two-column loads in FP64, where the layout admits them: 172.7
        // against 165.8 GLUP/s at 256^3, 190.0 against 183.7 at 512^3; in
        // FP32 they gained nothing, 259.5 / 296.7 against 258.8 / 307.0)
        return dtype == 0 ? fused_q1_3_t<double, 64, 16, 512, 4>(g, src, dst, b, h2, s, src_pairs)
                          : fused_q1_3_t<float, 64, 16, 256, 2>(g, src, dst, b, h2, s, false);
    return dtype == 0 ? fused_fd3_t<double, 64, 16, 512, 1>(g, src, dst, b, h2, s)
                      : fused_fd3_t<float, 64, 16, 512, 1>(g, src, dst, b, h2, s);
}

}  // namespace cs
