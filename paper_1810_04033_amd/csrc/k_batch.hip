// Batched patches: many independent Dirichlet patches of block-structured
// meshes (Sec. 1 and Sec. 2: regular patches of adaptive meshes) swept by one
// launch per sweep for all patches of a group.
//
// A group holds patches of one stencil, element type and tile variant.  Its
// device table lists every patch's geometry, arrays and the first index of
// its work items; a workgroup finds its patch by binary search over those
// prefixes (the table read is uniform across the workgroup) and then runs the
// same tile body as the single-grid fused kernels.  Patches are sorted by size,
// largest first, so the hardware dispatcher hands out the longest work first.
// The sweeps ping-pong between each patch's u and its work array tmp.
//
// Per-patch residual norms come from a fixed decomposition of each patch into
// row blocks (it depends on the patch's own shape only) and a per-patch
// finisher that folds its partials in order, so a patch's norms do not depend
// on which other patches share the batch.
#include "cs_tiles.h"

#include "cs_batch.h"

namespace cs {

namespace {

// which prefix a launch's items follow
enum { kItemsSweep = 0, kItemsRows = 1, kItemsHalo = 2 };

__device__ inline int find_patch(const BatchPatch* __restrict__ tab, int count, int64_t w, int kind)
{
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        const int64_t beg = kind == kItemsRows ? tab[mid].res_begin
                                               : (kind == kItemsHalo ? tab[mid].halo_begin : tab[mid].item_begin);
        if (beg <= w)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

template <typename T, int TX, int TY, int NT, int D>
__global__ void __launch_bounds__(NT)
k_batch_fd3(const BatchPatch* __restrict__ tab, int count, int phase)
{
    const int64_t w = blockIdx.x;
    const int p = find_patch(tab, count, w, kItemsSweep);
    const BatchPatch P = tab[p];
    const TileBox tb = tile_box<TX, TY>(P.g, P.tiles_x, P.tiles_y, P.chunks, w - P.item_begin);
    const T* src = (const T*)(phase ? P.tmp : P.u);
    T* dst = (T*)(phase ? P.u : P.tmp);
    fd3_tile<T, TX, TY, NT, D>(src, dst, (const T*)P.b, P.g, (T)P.h2, tb);
}

// Two red-black sweeps per launch (the large 7-point tile class).
template <typename T, int TX, int TY, int NT, int D, int NB>
__global__ void __launch_bounds__(NT)
k_batch_fd3_two(const BatchPatch* __restrict__ tab, int count, int phase)
{
    const int64_t w = blockIdx.x;
    const int p = find_patch(tab, count, w, kItemsSweep);
    const BatchPatch P = tab[p];
    const TileBox tb = tile_box<TX, TY>(P.g, P.tiles_x, P.tiles_y, P.chunks, w - P.item_begin);
    const T* src = (const T*)(phase ? P.tmp : P.u);
    T* dst = (T*)(phase ? P.u : P.tmp);
    fd3_tile_two<T, TX, TY, NT, D, NB>(src, dst, (const T*)P.b, P.g, (T)P.h2, tb);
}

template <typename T, int TX, int TY, int NT, int WPE, bool ROWWISE>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WPE)))
k_batch_q1_3(const BatchPatch* __restrict__ tab, int count, int phase)
{
    const int64_t w = blockIdx.x;
    const int p = find_patch(tab, count, w, kItemsSweep);
    const BatchPatch P = tab[p];
    const TileBox tb = tile_box<TX, TY>(P.g, P.tiles_x, P.tiles_y, P.chunks, w - P.item_begin);
    const T* src = (const T*)(phase ? P.tmp : P.u);
    T* dst = (T*)(phase ? P.u : P.tmp);
    q1_3_tile_pairs<T, TX, TY, NT, ROWWISE>(src, dst, (const T*)P.b, P.g, (T)P.h2, tb);
}

// All sweeps of a small patch in one workgroup with the patch resident in
// LDS: the halo'd box of u is loaded once, every colour phase updates its
// points in place in LDS with a workgroup barrier after it, and the interior
// goes back to u after the last sweep -- one launch and one trip through HBM
// for all sweeps.  A phase is one colour for red-black and, for the 27-point
// stencil, the two colours {2m, 2m+1}, which differ only in x parity and so
// never read each other (zero face weights): running them together is
// running them one after the other.  Each thread keeps the LDS offsets and the
// right-hand-side values of its points of every phase in registers (at most
// PMAX per phase; the host admits only patches that fit).  The point update is
// the colour pass's, so the iterate equals the colour passes' bit for bit.
template <typename T, int ST, int NT, int CAP, int PMAX>
__global__ void __launch_bounds__(NT)
k_batch_resident(const BatchPatch* __restrict__ tab, int nsweeps)
{
    constexpr int NPH = ST == FD ? 2 : 4;
    __shared__ T L[CAP];
    const BatchPatch P = tab[blockIdx.x];
    const Geo& g = P.g;
    const int nx = (int)g.nx, ny = (int)g.ny, nz = (int)g.nz;
    const int wx = nx + 2, lsz = wx * (ny + 2), total = lsz * (nz + 2);
    T* u = (T*)P.u;
    const T* __restrict__ b = (const T*)P.b;
    const int tid = threadIdx.x;
    for (int t = tid; t < total; t += NT) {
        const int k = t / lsz, r = t - k * lsz, j = r / wx, i = r - j * wx;
        L[t] = u[k * g.sz + j * g.sy + i];
    }
    int off[NPH][PMAX];
    T bv[NPH][PMAX];
#pragma unroll
    for (int ph = 0; ph < NPH; ++ph) {
#pragma unroll
        for (int sl = 0; sl < PMAX; ++sl) {
            const int w = tid + NT * sl;
            int i = 0, j = 0, k = 0;
            bool ok;
            if (ST == FD) {
                const int cx = (nx + 1) / 2;
                ok = w < cx * ny * nz;
                if (ok) {
                    const int m = w % cx, row = w / cx;
                    j = 1 + row % ny;
                    k = 1 + row / ny;
                    i = 1 + ((ph + (j - 1) + (k - 1) + g.parity) & 1) + 2 * m;
                    ok = i <= nx;
                }
            } else {
                const int j0 = 1 + (((ph & 1) + g.parity) & 1);
                const int k0 = 1 + (((ph >> 1) + g.parity) & 1);
                const int ry = (ny - j0) / 2 + 1, rz = (nz - k0) / 2 + 1;
                ok = j0 <= ny && k0 <= nz && w < nx * ry * rz;
                if (ok) {
                    i = 1 + w % nx;
                    j = j0 + 2 * ((w / nx) % ry);
                    k = k0 + 2 * (w / (nx * ry));
                }
            }
            off[ph][sl] = ok ? k * lsz + j * wx + i : -1;
            bv[ph][sl] = ok ? b[k * g.sz + j * g.sy + i] : T(0);
        }
    }
    __syncthreads();
    const T h2 = (T)P.h2;
    for (int sw = 0; sw < nsweeps; ++sw) {
#pragma unroll
        for (int ph = 0; ph < NPH; ++ph) {
#pragma unroll
            for (int sl = 0; sl < PMAX; ++sl) {
                int q = off[ph][sl];
                if (q < 0) continue;
                T bq = bv[ph][sl];
                // opaque to the compiler, so it does not hoist each point's
                // neighbour addresses and h^2 b out of the sweep loop (that
                // keeps them all live at once and spills)
                asm volatile("" : "+v"(q), "+v"(bq));
                auto ld = [&](int ox, int oy, int oz) { return L[q + oz * lsz + oy * wx + ox]; };
                L[q] = gs_value<T, 3, ST>(h2, bq, ld);
            }
            __syncthreads();
        }
    }
    const int inner = nx * ny * nz;
    for (int t = tid; t < inner; t += NT) {
        const int i = 1 + t % nx, row = t / nx, j = 1 + row % ny, k = 1 + row / ny;
        u[k * g.sz + j * g.sy + i] = L[k * lsz + j * wx + i];
    }
}

// Patches whose whole halo'd cross-section fits several times in LDS: one
// workgroup per patch streams through z with S sweeps per pass, in place in
// u.  Sweep j trails sweep j-1 by two planes, in the order of the colour
// passes:
//   7-point, step t:   R_j on plane t-2j, then B_j on plane t-2j-1, j = 0..S-1
//   27-point, step t:  A_j, B_j on plane t-2j, then C_j, D_j on plane t-2j-1
// (t runs over all planes for 7 points, over the "even" planes, two per step,
// for 27 points; A..D are the four row phases).  Every update reads the values
// the colour passes give it: the neighbour plane t-2j+1 already holds sweep
// j-1 (its last phase ran earlier in the step), the plane t-2j-1 still holds
// sweep j-1 (sweep j reaches it later).  The tile is the whole cross-section,
// so nothing is recomputed.  A window of 2S+1+NPL planes (NPL planes per step)
// lives in LDS slots, the planes leaving it are final and go back to u, and
// the planes entering it are old ones (the pass has not written them).  Passes
// repeat until nsweeps sweeps are done.  Each thread owns pairs of columns of
// opposite classes ((x, x+1) in row-major order for 7 points, rows (y, y+1) at
// one x for 27 points), so every phase gives it one point per pair; the
// right-hand side of its columns rides in a shift register of planes.  Point
// updates are the colour pass's, so the iterate equals the colour passes' bit
// for bit.
template <typename T, int ST, int NT, int CAP, int SMAX, int PP, int MPL>
__global__ void __launch_bounds__(NT)
k_batch_planes(const BatchPatch* __restrict__ tab, int nsweeps)
{
    constexpr int NPL = ST == FD ? 1 : 2;      // planes per step
    constexpr int RB = NPL + 2 * SMAX - 1;     // b register: ring[d] = plane t + NPL - 1 - d
    __shared__ __attribute__((aligned(16))) T L[CAP];
    const BatchPatch P = tab[blockIdx.x];
    const Geo& g = P.g;
    const int nx = (int)g.nx, ny = (int)g.ny, nz = (int)g.nz;
    const int wx = nx + 2, PL = wx * (ny + 2);
    int smax = (CAP / PL - 1 - NPL) / 2;
    if (smax > SMAX) smax = SMAX;
    T* u = (T*)P.u;
    const T* __restrict__ b = (const T*)P.b;
    const T h2 = (T)P.h2;
    const int tid = threadIdx.x;
    const int par = g.parity;

    // column pairs: LDS and global in-plane offsets and the class of each
    // column (7 points: (x-1)+(y-1)+parity; 27 points: the row type)
    int lo[PP][2], go[PP][2], cls[PP][2];
#pragma unroll
    for (int q = 0; q < PP; ++q) {
        const int pi = tid + NT * q;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            int x, y;
            bool ok;
            if (ST == FD) {
                const int c = 2 * pi + h;
                ok = c < nx * ny;
                x = 1 + (ok ? c % nx : 0);
                y = 1 + (ok ? c / nx : 0);
            } else {
                ok = pi < nx * ((ny + 1) / 2);
                x = 1 + (ok ? pi % nx : 0);
                y = 1 + (ok ? 2 * (pi / nx) + h : 0);
                ok = ok && y <= ny;
            }
            lo[q][h] = ok ? y * wx + x : -1;
            go[q][h] = ok ? (int)(y * g.sy + x) : 0;
            cls[q][h] = ST == FD ? (((x - 1) + (y - 1) + par) & 1) : ((y - 1 + par) & 1);
        }
    }
    int goff[MPL];
#pragma unroll
    for (int m = 0; m < MPL; ++m) {
        const int t = tid + NT * m;
        const int y = t / wx;
        goff[m] = t < PL ? (int)(y * g.sy + (t - y * wx)) : -1;
    }
    // (the offsets go through an empty asm so that their 64-bit addresses are
    // formed where used instead of being kept live across the step loop)
    auto load_plane = [&](int k, T* v) {
        const bool kin = k >= 0 && k <= nz + 1;
        const T* sp = u + (kin ? k : 0) * g.sz;
#pragma unroll
        for (int m = 0; m < MPL; ++m) {
            int o = goff[m];
            asm volatile("" : "+v"(o));
            v[m] = (kin && o >= 0) ? sp[o] : T(0);
        }
    };
    auto load_b = [&](int k, T (&v)[PP][2]) {
        const bool kin = k >= 1 && k <= nz;
        const T* bp = b + (kin ? k : 0) * g.sz;
#pragma unroll
        for (int q = 0; q < PP; ++q)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                int o = go[q][h];
                asm volatile("" : "+v"(o));
                v[q][h] = (kin && lo[q][h] >= 0) ? bp[o] : T(0);
            }
    };
    auto is_even = [&](int k) { return ((k - 1 + par) & 1) == 0; };

    T ring[PP][2][RB];
    for (int done = 0; done < nsweeps;) {
        const int S = nsweeps - done < smax ? nsweeps - done : smax;
        const int NS = 2 * S + 1 + NPL;
        // slot of plane p = p mod NS, formed from the current step's slot
        // (a modulo by a run-time NS costs a long scalar sequence per call,
        // repeated by every wave); planes lie within NS of the step's plane
        const int t0 = ST == FD ? 1 : (is_even(1) ? 1 : 2);
        int tcur = t0, sbase = t0 % NS;
        auto slot = [&](int p) -> T* {
            int k = sbase + (p - tcur);
            k += k < 0 ? NS : 0;
            k -= k >= NS ? NS : 0;
            return L + k * PL;
        };
        auto store_plane = [&](const T* v, int p) {
            T* lp = slot(p);
#pragma unroll
            for (int m = 0; m < MPL; ++m) {
                const int t = tid + NT * m;
                if (t < PL) lp[t] = v[m];
            }
        };
        auto write_plane = [&](int p) {
            if (p < 1 || p > nz) return;
            const T* lp = slot(p);
            T* dp = u + p * g.sz;
#pragma unroll
            for (int q = 0; q < PP; ++q)
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    int o = go[q][h], l = lo[q][h];
                    asm volatile("" : "+v"(o), "+v"(l));
                    if (l >= 0) dp[o] = lp[l];
                }
        };
        // the thread's points of class `sel` on plane p, b from rb: the two
        // columns of a pair have opposite classes, so each pair gives exactly
        // one point, picked by a select rather than a branch per column (a
        // divergent branch per column costs a run of scalar mask instructions
        // in every wave, and the scalar unit is shared by the CU)
        auto phase = [&](int p, int sel, const T (&rb)[PP][2]) {
            if (p < 1 || p > nz) return;
            const T* lm = slot(p - 1);
            T* lk = slot(p);
            const T* lq = slot(p + 1);
#pragma unroll
            for (int q = 0; q < PP; ++q) {
                const bool first = cls[q][0] == sel;
                // opaque, so neither the selected offset nor the neighbour
                // addresses are hoisted out of the step loop (all of them
                // live at once would spill)
                int l0 = lo[q][0], l1 = lo[q][1];
                asm volatile("" : "+v"(l0), "+v"(l1));
                int o = first ? l0 : l1;
                T bq = first ? rb[q][0] : rb[q][1];
                if (o < 0) continue;
                asm volatile("" : "+v"(o), "+v"(bq));
                auto ld = [&](int ox, int oy, int oz) {
                    const T* pl = oz < 0 ? lm : (oz > 0 ? lq : lk);
                    return pl[o + oy * wx + ox];
                };
                lk[o] = gs_value<T, 3, ST>(h2, bq, ld);
            }
        };
        const int t_last = nz + 2 * S - 1;
        // planes 0 .. t0+1-NPL straight into LDS, t0+2-NPL .. t0+1 into the
        // registers stored at the top of the first step
        {
            T v[MPL];
            for (int k = 0; k <= t0 + 1 - NPL; ++k) {
                load_plane(k, v);
                store_plane(v, k);
            }
        }
        T pre[NPL][MPL];
        T bnew[NPL][PP][2];
#pragma unroll
        for (int i = 0; i < NPL; ++i) load_plane(t0 + 2 - NPL + i, pre[i]);
#pragma unroll
        for (int d = 0; d < RB; ++d) {
            T tb[PP][2];
            load_b(t0 + NPL - 1 - d, tb);
#pragma unroll
            for (int q = 0; q < PP; ++q)
#pragma unroll
                for (int h = 0; h < 2; ++h) ring[q][h][d] = tb[q][h];
        }
        for (int t = t0; t <= t_last; t += NPL) {
#pragma unroll
            for (int i = 0; i < NPL; ++i)
                if (t + 2 - NPL + i <= nz + 1) store_plane(pre[i], t + 2 - NPL + i);
            const bool more = t + NPL <= t_last;
            if (more) {
#pragma unroll
                for (int i = 0; i < NPL; ++i) {
                    load_plane(t + 2 + i, pre[i]);
                    load_b(t + 2 * NPL - 1 - i, bnew[i]);
                }
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < SMAX; ++j) {
                if (j < S) {
                    T r0[PP][2], r1[PP][2];
#pragma unroll
                    for (int q = 0; q < PP; ++q)
#pragma unroll
                        for (int h = 0; h < 2; ++h) {
                            r0[q][h] = ring[q][h][NPL - 1 + 2 * j];  // plane t - 2j
                            r1[q][h] = ring[q][h][NPL + 2 * j];      // plane t - 2j - 1
                        }
                    const int p0 = t - 2 * j, p1 = t - 2 * j - 1;
                    if (ST == FD) {
                        phase(p0, (p0 - 1) & 1, r0);  // red of plane p0
                        __syncthreads();
                        phase(p1, p1 & 1, r1);        // black of plane p1
                        __syncthreads();
                    } else {
                        phase(p0, 0, r0);             // A
                        __syncthreads();
                        phase(p0, 1, r0);             // B
                        __syncthreads();
                        phase(p1, 0, r1);             // C
                        __syncthreads();
                        phase(p1, 1, r1);             // D
                        __syncthreads();
                    }
                }
            }
            // planes finished by the last sweep of the pass
            if (ST == FD) {
                write_plane(t - 2 * S + 1);
            } else {
                write_plane(t - 2 * S + 2);
                write_plane(t - 2 * S + 1);
            }
            if (more) {
#pragma unroll
                for (int q = 0; q < PP; ++q)
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
#pragma unroll
                        for (int d = RB - 1; d >= NPL; --d) ring[q][h][d] = ring[q][h][d - NPL];
#pragma unroll
                        for (int i = 0; i < NPL; ++i) ring[q][h][i] = bnew[i][q][h];
                    }
            }
            tcur += NPL;
            sbase += NPL;
            sbase -= sbase >= NS ? NS : 0;
        }
        done += S;
        // the next pass reads back what this one wrote
        __threadfence_block();
        __syncthreads();
    }
}

// Halo copy u -> tmp, one workgroup per plane k of a patch (nz + 2 items):
// the whole plane for k = 0 and k = nz + 1, else its two halo rows and two
// halo columns.
template <typename T>
__global__ void __launch_bounds__(256) k_batch_halo(const BatchPatch* __restrict__ tab, int count)
{
    const int64_t w = blockIdx.x;
    const int p = find_patch(tab, count, w, kItemsHalo);
    const BatchPatch P = tab[p];
    const Geo& g = P.g;
    const int k = (int)(w - P.halo_begin);
    const T* src = (const T*)P.u + (int64_t)k * g.sz;
    T* dst = (T*)P.tmp + (int64_t)k * g.sz;
    const int nx = (int)g.nx, ny = (int)g.ny, wx = nx + 2, sy = (int)g.sy;
    if (k == 0 || k == g.nz + 1) {
        const int total = wx * (ny + 2);
        for (int t = threadIdx.x; t < total; t += 256) {
            const int j = t / wx, i = t - j * wx;
            dst[j * sy + i] = src[j * sy + i];
        }
        return;
    }
    const int total = 2 * wx + 2 * ny;
    for (int t = threadIdx.x; t < total; t += 256) {
        int i, j;
        if (t < 2 * wx) {
            j = t < wx ? 0 : ny + 1;
            i = t < wx ? t : t - wx;
        } else {
            const int r = t - 2 * wx;
            j = 1 + (r >> 1);
            i = (r & 1) ? nx + 1 : 0;
        }
        dst[j * sy + i] = src[j * sy + i];
    }
}

constexpr int kRowsPerItem = 16;

// Row-block items (residual and copy-back): item covers kRowsPerItem rows
// (j, k) of the patch interior; 256 threads = 64 along x x 4 rows.
template <typename T>
__global__ void __launch_bounds__(256) k_batch_copyback(const BatchPatch* __restrict__ tab, int count)
{
    const int64_t w = blockIdx.x;
    const int p = find_patch(tab, count, w, kItemsRows);
    const BatchPatch P = tab[p];
    const Geo& g = P.g;
    const int64_t item = w - P.res_begin;
    const int64_t rows = g.ny * g.nz;
    const T* src = (const T*)P.tmp;
    T* dst = (T*)P.u;
    for (int rr = threadIdx.y; rr < kRowsPerItem; rr += 4) {
        const int64_t row = item * kRowsPerItem + rr;
        if (row >= rows) break;
        const int64_t j = 1 + row % g.ny, k = 1 + row / g.ny;
        for (int64_t i = 1 + threadIdx.x; i <= g.nx; i += 64) {
            const int64_t q = k * g.sz + j * g.sy + i;
            dst[q] = src[q];
        }
    }
}

// One patch's norms from its n row-block partials, by a 64-thread
// workgroup: lane l folds partials l, l + 64, l + 128, ... in order, then
// the 64 lane values are added by a fixed binary tree.  The order depends
// only on n, so a patch's norms do not depend on the rest of the batch.
__device__ inline void fold_partials(const Partial* __restrict__ ps, int n, double* __restrict__ out)
{
    __shared__ double sh[3][64];
    const int l = threadIdx.x;
    double a = 0.0, m = 0.0, c = 0.0;
    for (int i = l; i < n; i += 64) {
        const Partial q = ps[i];
        a += q.sum_r2;
        m = fmax(m, q.max_r);
        c += q.sum_b2;
    }
    sh[0][l] = a;
    sh[1][l] = m;
    sh[2][l] = c;
    __syncthreads();
    for (int w = 32; w > 0; w >>= 1) {
        if (l < w) {
            sh[0][l] = sh[0][l] + sh[0][l + w];
            sh[1][l] = fmax(sh[1][l], sh[1][l + w]);
            sh[2][l] = sh[2][l] + sh[2][l + w];
        }
        __syncthreads();
    }
    if (l == 0) {
        out[0] = sqrt(sh[0][0]);
        out[1] = sh[1][0];
        out[2] = sqrt(sh[2][0]);
    }
}

// Groups too small to fill the device with tiles: one colour phase of every
// patch per launch, in place in u (a phase is one colour for red-black, an
// x-parity pair of colours for 27 points, which never read each other), so a
// patch spreads over many workgroups whatever its size.  An item covers
// kColRows rows (j, k) of the phase, 64 threads along x x 4 rows.  The point
// update is the colour pass's, so the iterate equals it bit for bit.
constexpr int kColRows = 8;

template <typename T, int ST>
__global__ void __launch_bounds__(256)
k_batch_colour(const BatchPatch* __restrict__ tab, int count, int phase)
{
    const int64_t w = blockIdx.x;
    const int p = find_patch(tab, count, w, kItemsSweep);
    const BatchPatch P = tab[p];
    const Geo& g = P.g;
    const int64_t item = w - P.item_begin;
    T* u = (T*)P.u;
    const T* b = (const T*)P.b;
    const T h2 = (T)P.h2;
    const int par = g.parity;
    // rows of the phase: every row for red-black, for 27 points the rows whose
    // y and z parities are the phase's (py = phase & 1, pz = phase >> 1)
    const int64_t jo = ST == FD ? 0 : ((phase & 1) + par) & 1;
    const int64_t ko = ST == FD ? 0 : ((phase >> 1) + par) & 1;
    const int64_t rows_y = ST == FD ? g.ny : (g.ny - jo + 1) / 2;
    const int64_t rows = rows_y * (ST == FD ? g.nz : (g.nz - ko + 1) / 2);
    const int64_t sy = g.sy, sz = g.sz;
    for (int rr = threadIdx.y; rr < kColRows; rr += 4) {
        const int64_t row = item * kColRows + rr;
        if (row >= rows) break;
        const int64_t ty = row % rows_y, tz = row / rows_y;
        const int64_t j = ST == FD ? 1 + ty : 1 + jo + 2 * ty;
        const int64_t k = ST == FD ? 1 + tz : 1 + ko + 2 * tz;
        // red-black: points with (i-1)+(j-1)+(k-1)+parity = phase (mod 2)
        const int64_t i0 = ST == FD ? 1 + ((phase + (j - 1) + (k - 1) + par) & 1) : 1;
        const int64_t di = ST == FD ? 2 : 1;
        for (int64_t i = i0 + di * threadIdx.x; i <= g.nx; i += di * 64) {
            const int64_t q = k * sz + j * sy + i;
            auto ld = [&](int ox, int oy, int oz) { return u[q + oz * sz + oy * sy + ox]; };
            u[q] = gs_value<T, 3, ST>(h2, b[q], ld);
        }
    }
}

template <typename S, int ST>
__global__ void __launch_bounds__(256)
k_batch_residual(const BatchPatch* __restrict__ tab, int count, Partial* __restrict__ partials)
{
    __shared__ double sh[3 * 256];
    const int64_t w = blockIdx.x;
    const int p = find_patch(tab, count, w, kItemsRows);
    const BatchPatch P = tab[p];
    const Geo& g = P.g;
    const int64_t item = w - P.res_begin;
    const int64_t rows = g.ny * g.nz;
    const S* u = (const S*)P.u;
    const S* b = (const S*)P.b;
    const int64_t sy = g.sy, sz = g.sz;
    double s_r2 = 0.0, mx = 0.0, s_b2 = 0.0;
    for (int rr = threadIdx.y; rr < kRowsPerItem; rr += 4) {
        const int64_t row = item * kRowsPerItem + rr;
        if (row >= rows) break;
        const int64_t j = 1 + row % g.ny, k = 1 + row / g.ny;
        for (int64_t i = 1 + threadIdx.x; i <= g.nx; i += 64) {
            const int64_t q = k * g.sz + j * g.sy + i;
            auto ld = [&](int ox, int oy, int oz) { return (double)u[q + oz * sz + oy * sy + ox]; };
            const double su = ordered_sum<double, 3, ST, true>(ld);
            const double bq = (double)b[q];
            const double rq = bq - su / P.hh;
            s_r2 += rq * rq;
            s_b2 += bq * bq;
            mx = fmax(mx, fabs(rq));
        }
    }
    const int t = threadIdx.y * 64 + threadIdx.x;
    sh[t] = s_r2;
    sh[256 + t] = mx;
    sh[512 + t] = s_b2;
    __syncthreads();
    for (int wdt = 128; wdt > 0; wdt >>= 1) {
        if (t < wdt) {
            sh[t] = sh[t] + sh[t + wdt];
            sh[256 + t] = fmax(sh[256 + t], sh[256 + t + wdt]);
            sh[512 + t] = sh[512 + t] + sh[512 + t + wdt];
        }
        __syncthreads();
    }
    if (t == 0) {
        partials[w].sum_r2 = sh[0];
        partials[w].max_r = sh[256];
        partials[w].sum_b2 = sh[512];
    }
}

// One workgroup per patch folds the patch's partials in order.
__global__ void __launch_bounds__(64)
k_batch_finish(const BatchPatch* __restrict__ tab, const Partial* __restrict__ partials,
               double* __restrict__ norms)
{
    const BatchPatch P = tab[blockIdx.x];
    fold_partials(partials + P.res_begin, P.res_items, norms + 3 * P.index);
}

// ---- batched refinement steps ---------------------------------------------

__device__ inline int find_ir(const IrPatch* __restrict__ tab, int count, int64_t w)
{
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tab[mid].res_begin <= w)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// The smallest power of two >= v (1 for v <= 0 or not finite), exactly:
// a positive finite double is a power of two iff its significand field is
// zero (normal) or a single bit (subnormal); otherwise the next one up is
// formed from the exponent (or the leading significand bit) alone.
__device__ inline double pow2_at_least(double v)
{
    if (!(v > 0.0) || !(v <= 1.7976931348623157e308)) return 1.0;
    const unsigned long long bits = (unsigned long long)__double_as_longlong(v);
    const unsigned long long man = bits & ((1ull << 52) - 1);
    const unsigned ex = (unsigned)(bits >> 52) & 0x7ffu;
    if (ex == 0) {  // subnormal: v = man * 2^-1074
        const unsigned long long p = 1ull << (63 - __clzll((long long)man));
        return __longlong_as_double((long long)(man == p ? man : p << 1));
    }
    if (man == 0) return v;
    return __longlong_as_double((long long)((unsigned long long)(ex + 1) << 52));
}

template <int ST>
__device__ __forceinline__ void ir_rows(const IrPatch& P, int64_t item, double inv, double& s_r2,
                                        double& mx, double& s_b2)
{
    const Geo& g = P.g;
    const int64_t rows = g.ny * g.nz, sy = g.sy, sz = g.sz;
    for (int rr = threadIdx.y; rr < kRowsPerItem; rr += 4) {
        const int64_t row = item * kRowsPerItem + rr;
        if (row >= rows) break;
        const int64_t j = 1 + row % g.ny, k = 1 + row / g.ny;
        for (int64_t i = 1 + threadIdx.x; i <= g.nx; i += 64) {
            const int64_t q = k * sz + j * sy + i;
            const int64_t q2 = k * P.g2.sz + j * P.g2.sy + i;
            auto ld = [&](int ox, int oy, int oz) { return P.x[q + oz * sz + oy * sy + ox]; };
            const double su = ordered_sum<double, 3, ST, true>(ld);
            const double bq = P.b[q];
            const double rq = bq - su / P.hh;
            P.r32[q2] = (float)(rq * inv);
            P.e[q2] = 0.0f;
            s_r2 += rq * rq;
            s_b2 += bq * bq;
            mx = fmax(mx, fabs(rq));
        }
    }
}

__global__ void __launch_bounds__(256)
k_batch_ir_residual(const IrPatch* __restrict__ tab, int count, const double* norms,
                    double* __restrict__ scales, Partial* __restrict__ partials)
{
    __shared__ double sh[3 * 256];
    const int64_t w = blockIdx.x;
    const IrPatch P = tab[find_ir(tab, count, w)];
    const int64_t item = w - P.res_begin;
    // the scale of this step from the previous residual's max |r|
    const double sc = pow2_at_least(norms[3 * P.row + 1]);
    if (item == 0 && threadIdx.x == 0 && threadIdx.y == 0) scales[P.row] = sc;
    const double inv = 1.0 / sc;  // exact: sc is a power of two
    double s_r2 = 0.0, mx = 0.0, s_b2 = 0.0;
    if (P.stencil == FD)
        ir_rows<FD>(P, item, inv, s_r2, mx, s_b2);
    else
        ir_rows<Q1>(P, item, inv, s_r2, mx, s_b2);
    const int t = threadIdx.y * 64 + threadIdx.x;
    sh[t] = s_r2;
    sh[256 + t] = mx;
    sh[512 + t] = s_b2;
    __syncthreads();
    for (int wdt = 128; wdt > 0; wdt >>= 1) {
        if (t < wdt) {
            sh[t] = sh[t] + sh[t + wdt];
            sh[256 + t] = fmax(sh[256 + t], sh[256 + t + wdt]);
            sh[512 + t] = sh[512 + t] + sh[512 + t + wdt];
        }
        __syncthreads();
    }
    if (t == 0) {
        partials[w].sum_r2 = sh[0];
        partials[w].max_r = sh[256];
        partials[w].sum_b2 = sh[512];
    }
}

__global__ void __launch_bounds__(64)
k_batch_ir_finish(const IrPatch* __restrict__ tab, const Partial* __restrict__ partials,
                  double* __restrict__ norms)
{
    const IrPatch P = tab[blockIdx.x];
    fold_partials(partials + P.res_begin, P.res_items, norms + 3 * P.row);
}

__global__ void __launch_bounds__(256)
k_batch_ir_update(const IrPatch* __restrict__ tab, int count, const double* __restrict__ scales)
{
    const int64_t w = blockIdx.x;
    const IrPatch P = tab[find_ir(tab, count, w)];
    const int64_t item = w - P.res_begin;
    const Geo& g = P.g;
    const double sc = scales[P.row];
    const int64_t rows = g.ny * g.nz;
    for (int rr = threadIdx.y; rr < kRowsPerItem; rr += 4) {
        const int64_t row = item * kRowsPerItem + rr;
        if (row >= rows) break;
        const int64_t j = 1 + row % g.ny, k = 1 + row / g.ny;
        for (int64_t i = 1 + threadIdx.x; i <= g.nx; i += 64) {
            const int64_t q = k * g.sz + j * g.sy + i;
            const int64_t q2 = k * P.g2.sz + j * P.g2.sy + i;
            P.x[q] = P.x[q] + (double)P.e[q2] * sc;
        }
    }
}

}  // namespace

cs_status launch_batch_ir_residual(const IrPatch* tab, int count, int64_t items, Partial* partials,
                                   double* scales, double* norms, hipStream_t s)
{
    if (count <= 0 || items <= 0) return CS_OK;
    hipLaunchKernelGGL(k_batch_ir_residual, dim3((unsigned)items), dim3(64, 4), 0, s, tab, count,
                       (const double*)norms, scales, partials);
    cs_status st = check_launch("batched refinement residual");
    if (st != CS_OK) return st;
    hipLaunchKernelGGL(k_batch_ir_finish, dim3(count), dim3(64), 0, s, tab, partials, norms);
    return check_launch("batched refinement residual finish");
}

cs_status launch_batch_ir_update(const IrPatch* tab, int count, int64_t items, const double* scales,
                                 hipStream_t s)
{
    if (count <= 0 || items <= 0) return CS_OK;
    hipLaunchKernelGGL(k_batch_ir_update, dim3((unsigned)items), dim3(64, 4), 0, s, tab, count, scales);
    return check_launch("batched refinement update");
}

int64_t batch_residual_items(const Geo& g)
{
    return (g.ny * g.nz + kRowsPerItem - 1) / kRowsPerItem;
}

// Tile of each variant: (TX, TY) used to count a patch's work items.
void batch_variant_tile(int stencil, int variant, int* tx, int* ty)
{
    static const int fd[3][2] = {{16, 16}, {32, 16}, {64, 16}};
    static const int q1[3][2] = {{16, 8}, {32, 16}, {64, 16}};
    const int v = variant < 0 ? 0 : (variant > 2 ? 2 : variant);
    *tx = stencil == FD ? fd[v][0] : q1[v][0];
    *ty = stencil == FD ? fd[v][1] : q1[v][1];
}

bool batch_variant_pairs(int stencil, int variant)
{
    return stencil == FD && variant >= 2;
}

cs_status launch_batch_sweep(int dtype, int stencil, int variant, const BatchPatch* tab, int count,
                             int64_t items, int phase, bool two, hipStream_t s)
{
    if (items <= 0) return CS_OK;
    const dim3 grid((unsigned)items);
    if (two) {
        if (!batch_variant_pairs(stencil, variant)) {
            set_error("no double sweep for this tile variant");
            return CS_EUNSUPPORTED;
        }
        if (dtype == 0)
            hipLaunchKernelGGL((k_batch_fd3_two<double, 64, 16, 1024, 2, 2>), grid, dim3(1024), 0,
                               s, tab, count, phase);
        else
            hipLaunchKernelGGL((k_batch_fd3_two<float, 64, 16, 1024, 2, 2>), grid, dim3(1024), 0,
                               s, tab, count, phase);
        return check_launch("batched double sweep");
    }
#define CS_BFD(T, TX, TY, NT, D) \
    hipLaunchKernelGGL((k_batch_fd3<T, TX, TY, NT, D>), grid, dim3(NT), 0, s, tab, count, phase)
#define CS_BQ1(T, TX, TY, NT, WPE, RW) \
    hipLaunchKernelGGL((k_batch_q1_3<T, TX, TY, NT, WPE, RW>), grid, dim3(NT), 0, s, tab, count, phase)
    if (stencil == FD) {
        if (dtype == 0) {
            if (variant == 0) CS_BFD(double, 16, 16, 256, 1);
            else if (variant == 1) CS_BFD(double, 32, 16, 256, 1);
            else CS_BFD(double, 64, 16, 512, 1);
        } else {
            if (variant == 0) CS_BFD(float, 16, 16, 256, 1);
            else if (variant == 1) CS_BFD(float, 32, 16, 256, 1);
            else CS_BFD(float, 64, 16, 512, 1);
        }
    } else {
        // the large FP64 tile and every FP32 tile take the row-wise pair
        // update (as the single-grid 27-point sweep)
        if (dtype == 0) {
            if (variant == 0) CS_BQ1(double, 16, 8, 128, 2, false);
            else if (variant == 1) CS_BQ1(double, 32, 16, 256, 2, false);
            else CS_BQ1(double, 64, 16, 512, 4, true);
        } else {
            if (variant == 0) CS_BQ1(float, 16, 8, 128, 2, true);
            else if (variant == 1) CS_BQ1(float, 32, 16, 256, 2, true);
            else CS_BQ1(float, 64, 16, 256, 2, true);
        }
    }
#undef CS_BFD
#undef CS_BQ1
    return check_launch("batched sweep");
}

// The two resident tiers: (threads, LDS elements, points per phase and
// thread).  Small: 512 threads and 6144 elements (a 16^3 patch with its
// halo); large: 1024 threads and up to 140.8 KB (FP64, a 24^3 patch) or
// 160 KB (FP32, a 32^3 patch) of LDS, one workgroup per CU.
namespace {
constexpr int kResSmallNT = 512, kResSmallCap = 6144;
constexpr int kResLargeNT = 1024, kResLargeCap64 = 17600, kResLargeCap32 = 40000;
template <int ST, bool F64, bool LARGE>
constexpr int res_pmax()
{
    return !LARGE ? (ST == FD ? 4 : 2) : (F64 ? (ST == FD ? 7 : 4) : (ST == FD ? 16 : 8));
}
bool res_fits(int stencil, const Geo& g, int nt, int cap, int pmax)
{
    const int64_t elems = (g.nx + 2) * (g.ny + 2) * (g.nz + 2);
    const int64_t per_phase = stencil == FD ? (g.nx + 1) / 2 * g.ny * g.nz
                                            : g.nx * ((g.ny + 1) / 2) * ((g.nz + 1) / 2);
    return elems <= cap && per_phase <= (int64_t)nt * pmax;
}
}  // namespace

int batch_resident_tier(int dtype, int stencil, const Geo& g)
{
    const bool f64 = dtype == 0;
    const int ps = stencil == FD ? res_pmax<FD, true, false>() : res_pmax<Q1, true, false>();
    if (res_fits(stencil, g, kResSmallNT, kResSmallCap, ps)) return 1;
    const int pl = f64 ? (stencil == FD ? res_pmax<FD, true, true>() : res_pmax<Q1, true, true>())
                       : (stencil == FD ? res_pmax<FD, false, true>() : res_pmax<Q1, false, true>());
    if (res_fits(stencil, g, kResLargeNT, f64 ? kResLargeCap64 : kResLargeCap32, pl)) return 2;
    return 0;
}

cs_status launch_batch_resident(int dtype, int stencil, int tier, const BatchPatch* tab, int count,
                                int nsweeps, hipStream_t s)
{
    if (count <= 0 || nsweeps <= 0) return CS_OK;
    const dim3 grid((unsigned)count);
#define CS_RES(T, ST, LARGE, CAP)                                                                 \
    hipLaunchKernelGGL((k_batch_resident<T, ST, LARGE ? kResLargeNT : kResSmallNT, CAP,          \
                                         res_pmax<ST, sizeof(T) == 8, LARGE>()>),               \
                       grid, dim3(LARGE ? kResLargeNT : kResSmallNT), 0, s, tab, nsweeps)
    if (tier == 1) {
        if (dtype == 0) {
            if (stencil == FD) CS_RES(double, FD, false, kResSmallCap);
            else CS_RES(double, Q1, false, kResSmallCap);
        } else {
            if (stencil == FD) CS_RES(float, FD, false, kResSmallCap);
            else CS_RES(float, Q1, false, kResSmallCap);
        }
    } else if (tier == 2) {
        if (dtype == 0) {
            if (stencil == FD) CS_RES(double, FD, true, kResLargeCap64);
            else CS_RES(double, Q1, true, kResLargeCap64);
        } else {
            if (stencil == FD) CS_RES(float, FD, true, kResLargeCap32);
            else CS_RES(float, Q1, true, kResLargeCap32);
        }
    } else {
        set_error("no resident tier %d", tier);
        return CS_EUNSUPPORTED;
    }
#undef CS_RES
    return check_launch("batched resident sweeps");
}

// The plane-streaming tier: 1024 threads, the whole LDS, at most 3 (7-point)
// or 2 (27-point) sweeps per pass and two column pairs per thread, taken where
// at least 2 sweeps fit.
namespace {
constexpr int kPlNT = 1024;
constexpr int pl_smax(int st) { return st == FD ? 3 : 2; }
constexpr int pl_pp(int) { return 2; }
constexpr int kPlCap64 = 20000, kPlCap32 = 40000;  // elements: 160 KB
constexpr int pl_mpl(int cap, int npl) { return (cap / (2 * 2 + 1 + npl) + kPlNT - 1) / kPlNT; }
}  // namespace

int batch_planes_sweeps(int dtype, int stencil, const Geo& g)
{
    const int npl = stencil == FD ? 1 : 2;
    const int64_t pl = (g.nx + 2) * (g.ny + 2);
    const int64_t cap = dtype == 0 ? kPlCap64 : kPlCap32;
    const int64_t s = (cap / pl - 1 - npl) / 2;
    const int smax = stencil == FD ? pl_smax(FD) : pl_smax(Q1);
    return (int)(s < smax ? s : smax);
}

// At most this many points: one workgroup carries the whole patch, so a much
// larger patch would make one long pole for the batch (a serving step waits
// for its slowest patch), while the tile kernels spread it over the device.
constexpr int64_t kPlMaxPoints = 1 << 17;

bool batch_planes_fits(int dtype, int stencil, const Geo& g)
{
    if (g.nx * g.ny * g.nz > kPlMaxPoints) return false;
    const int npl = stencil == FD ? 1 : 2;
    const int64_t pl = (g.nx + 2) * (g.ny + 2);
    const int64_t cap = dtype == 0 ? kPlCap64 : kPlCap32;
    const int64_t s = (cap / pl - 1 - npl) / 2;
    const int64_t pairs = stencil == FD ? (g.nx * g.ny + 1) / 2 : g.nx * ((g.ny + 1) / 2);
    return s >= 2 && pairs <= (int64_t)kPlNT * (stencil == FD ? pl_pp(FD) : pl_pp(Q1)) && g.nz >= 1;
}

// The small form: 512 threads, one column pair each, half the LDS, so two
// workgroups share a compute unit (for cross-sections of at most 1024 points,
// e.g. 32 x 32, whose pairs would leave half of a 1024-thread workgroup idle).
constexpr int kPlNTs = 512;
constexpr int kPlCap64s = 10000, kPlCap32s = 20000;  // elements: 80 KB
constexpr int pl_mpl_s(int cap, int npl) { return (cap / (2 * 2 + 1 + npl) + kPlNTs - 1) / kPlNTs; }

bool batch_planes_small(int dtype, int stencil, const Geo& g)
{
    const int npl = stencil == FD ? 1 : 2;
    const int64_t pl = (g.nx + 2) * (g.ny + 2);
    const int64_t cap = dtype == 0 ? kPlCap64s : kPlCap32s;
    int64_t s = (cap / pl - 1 - npl) / 2;
    const int smax = stencil == FD ? pl_smax(FD) : pl_smax(Q1);
    if (s > smax) s = smax;
    const int64_t pairs = stencil == FD ? (g.nx * g.ny + 1) / 2 : g.nx * ((g.ny + 1) / 2);
    // the same sweeps per pass as the large form
    return pairs <= kPlNTs && s == batch_planes_sweeps(dtype, stencil, g);
}

cs_status launch_batch_planes(int dtype, int stencil, const BatchPatch* tab, int count, int nsweeps,
                              hipStream_t s, bool small)
{
    if (count <= 0 || nsweeps <= 0) return CS_OK;
    if (small) {
        const dim3 grid((unsigned)count), blk(kPlNTs);
        if (dtype == 0) {
            if (stencil == FD)
                hipLaunchKernelGGL((k_batch_planes<double, FD, kPlNTs, kPlCap64s, pl_smax(FD), 1, pl_mpl_s(kPlCap64s, 1)>),
                                   grid, blk, 0, s, tab, nsweeps);
            else
                hipLaunchKernelGGL((k_batch_planes<double, Q1, kPlNTs, kPlCap64s, pl_smax(Q1), 1, pl_mpl_s(kPlCap64s, 2)>),
                                   grid, blk, 0, s, tab, nsweeps);
        } else {
            if (stencil == FD)
                hipLaunchKernelGGL((k_batch_planes<float, FD, kPlNTs, kPlCap32s, pl_smax(FD), 1, pl_mpl_s(kPlCap32s, 1)>),
                                   grid, blk, 0, s, tab, nsweeps);
            else
                hipLaunchKernelGGL((k_batch_planes<float, Q1, kPlNTs, kPlCap32s, pl_smax(Q1), 1, pl_mpl_s(kPlCap32s, 2)>),
                                   grid, blk, 0, s, tab, nsweeps);
        }
        return check_launch("batched plane-streaming sweeps");
    }
    const dim3 grid((unsigned)count), blk(kPlNT);
    if (dtype == 0) {
        if (stencil == FD)
            hipLaunchKernelGGL((k_batch_planes<double, FD, kPlNT, kPlCap64, pl_smax(FD), pl_pp(FD), pl_mpl(kPlCap64, 1)>),
                               grid, blk, 0, s, tab, nsweeps);
        else
            hipLaunchKernelGGL((k_batch_planes<double, Q1, kPlNT, kPlCap64, pl_smax(Q1), pl_pp(Q1), pl_mpl(kPlCap64, 2)>),
                               grid, blk, 0, s, tab, nsweeps);
    } else {
        if (stencil == FD)
            hipLaunchKernelGGL((k_batch_planes<float, FD, kPlNT, kPlCap32, pl_smax(FD), pl_pp(FD), pl_mpl(kPlCap32, 1)>),
                               grid, blk, 0, s, tab, nsweeps);
        else
            hipLaunchKernelGGL((k_batch_planes<float, Q1, kPlNT, kPlCap32, pl_smax(Q1), pl_pp(Q1), pl_mpl(kPlCap32, 2)>),
                               grid, blk, 0, s, tab, nsweeps);
    }
    return check_launch("batched plane-streaming sweeps");
}

cs_status launch_batch_halo(int dtype, const BatchPatch* tab, int count, int64_t halo_items, hipStream_t s)
{
    if (count <= 0 || halo_items <= 0) return CS_OK;
    if (halo_items > 0x7fffffff) { set_error("batch too large"); return CS_EUNSUPPORTED; }
    const dim3 grid((unsigned)halo_items);
    if (dtype == 0)
        hipLaunchKernelGGL(k_batch_halo<double>, grid, dim3(256), 0, s, tab, count);
    else
        hipLaunchKernelGGL(k_batch_halo<float>, grid, dim3(256), 0, s, tab, count);
    return check_launch("batched halo copy");
}

cs_status launch_batch_copyback(int dtype, const BatchPatch* tab, int count, int64_t res_items,
                                hipStream_t s)
{
    if (res_items <= 0) return CS_OK;
    if (dtype == 0)
        hipLaunchKernelGGL(k_batch_copyback<double>, dim3((unsigned)res_items), dim3(64, 4), 0, s,
                           tab, count);
    else
        hipLaunchKernelGGL(k_batch_copyback<float>, dim3((unsigned)res_items), dim3(64, 4), 0, s,
                           tab, count);
    return check_launch("batched copy back");
}

int64_t batch_colour_items(int stencil, const Geo& g)
{
    const int64_t rows = stencil == FD ? g.ny * g.nz : ((g.ny + 1) / 2) * ((g.nz + 1) / 2);
    return (rows + kColRows - 1) / kColRows;
}

cs_status launch_batch_colour(int dtype, int stencil, const BatchPatch* tab, int count, int64_t items,
                              int nsweeps, hipStream_t s)
{
    if (count <= 0 || items <= 0 || nsweeps <= 0) return CS_OK;
    if (items > 0x7fffffff) { set_error("colour group too large"); return CS_EUNSUPPORTED; }
    const dim3 grid((unsigned)items), blk(64, 4);
    const int nph = stencil == FD ? 2 : 4;
    for (int it = 0; it < nsweeps; ++it)
        for (int ph = 0; ph < nph; ++ph) {
            if (dtype == 0) {
                if (stencil == FD) hipLaunchKernelGGL((k_batch_colour<double, FD>), grid, blk, 0, s, tab, count, ph);
                else hipLaunchKernelGGL((k_batch_colour<double, Q1>), grid, blk, 0, s, tab, count, ph);
            } else {
                if (stencil == FD) hipLaunchKernelGGL((k_batch_colour<float, FD>), grid, blk, 0, s, tab, count, ph);
                else hipLaunchKernelGGL((k_batch_colour<float, Q1>), grid, blk, 0, s, tab, count, ph);
            }
            cs_status st = check_launch("batched colour pass");
            if (st != CS_OK) return st;
        }
    return CS_OK;
}

cs_status launch_batch_residual(int dtype, int stencil, const BatchPatch* tab, int count,
                                int64_t res_items, Partial* partials, double* norms, hipStream_t s)
{
    if (res_items <= 0) return CS_OK;
    const dim3 grid((unsigned)res_items), blk(64, 4);
    if (dtype == 0) {
        if (stencil == FD)
            hipLaunchKernelGGL((k_batch_residual<double, FD>), grid, blk, 0, s, tab, count, partials);
        else
            hipLaunchKernelGGL((k_batch_residual<double, Q1>), grid, blk, 0, s, tab, count, partials);
    } else {
        if (stencil == FD)
            hipLaunchKernelGGL((k_batch_residual<float, FD>), grid, blk, 0, s, tab, count, partials);
        else
            hipLaunchKernelGGL((k_batch_residual<float, Q1>), grid, blk, 0, s, tab, count, partials);
    }
    cs_status st = check_launch("batched residual");
    if (st != CS_OK) return st;
    hipLaunchKernelGGL(k_batch_finish, dim3(count), dim3(64), 0, s, tab, partials, norms);
    return check_launch("batched residual finish");
}

}  // namespace cs
