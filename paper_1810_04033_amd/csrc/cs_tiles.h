// Tile bodies of the fused Gauss-Seidel sweeps: every colour of one sweep in a single pass over
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
#pragma once

#include "cs_device.h"

#include <cstdint>
#include <type_traits>
#include "cs_internal.h"

namespace cs {

constexpr int kXcds = 8;

// Logical work index of this workgroup such that the hardware's round-robin
// placement of workgroups over the XCDs gives each XCD a contiguous range.
__device__ inline int64_t xcd_ordered_block(int64_t nblocks)
{
    const int64_t b = blockIdx.x;
    const int64_t per = nblocks / kXcds;
    const int64_t rem = nblocks % kXcds;
    const int64_t xcd = b % kXcds;
    const int64_t slot = b / kXcds;
    // XCDs [0, rem) hold per+1 blocks, the others per blocks
    const int64_t start = xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per;
    return start + slot;
}

// Work split of one grid: tile index (x fastest) and z chunk, planes split
// evenly over the chunks.
struct FusedWork {
    int tiles_x, tiles_y;
    int chunks;
    int64_t nblocks;
};

// The interior box a workgroup finalises: x from x0, y from y0 (tile T) and
// planes [z0, z1).
struct TileBox {
    int64_t x0, y0, z0, z1;
};

template <int TX, int TY>
__device__ inline TileBox tile_box(const Geo& g, int tiles_x, int tiles_y, int chunks, int64_t work)
{
    const int64_t tiles = (int64_t)tiles_x * tiles_y;
    const int64_t chunk = work / tiles;
    const int64_t tile = work % tiles;
    TileBox t;
    t.x0 = 1 + (tile % tiles_x) * TX;
    t.y0 = 1 + (tile / tiles_x) * TY;
    t.z0 = 1 + (chunk * g.nz) / chunks;
    t.z1 = 1 + ((chunk + 1) * g.nz) / chunks;
    return t;
}

template <typename T, int TX, int TY, int NT, int D>
struct FdCfg {
    static constexpr int W = TX + 4;           // region T+2, x extent
    static constexpr int HH = TY + 4;          // region T+2, y extent
    static constexpr int NCOL = W * HH;
    static constexpr int M = (NCOL + NT - 1) / NT;  // columns per thread
    // register planes k-2 .. k+1 in use plus D planes in flight
    static constexpr int RING = 4 + D;
};

// One red-black sweep of the 7-point stencil over the box tb, src -> dst.
template <typename T, int TX, int TY, int NT, int D>
__device__ __forceinline__ void fd3_tile(const T* __restrict__ src, T* __restrict__ dst,
                                         const T* __restrict__ b, const Geo& g, T h2,
                                         const TileBox& tb)
{
    using C = FdCfg<T, TX, TY, NT, D>;
    constexpr int W = C::W, M = C::M, NCOL = C::NCOL, R = C::RING;
    // two LDS buffer sets (planes k and k-1), alternating with the step parity,
    // so one barrier per plane step suffices
    __shared__ T lds[2][2][NCOL];
    // final values of plane k-1 (tile T only), written at step k and stored to
    // dst by whole rows at step k+1, alternating with the step parity
    __shared__ T lout[2][TX * TY];
    const int64_t x0 = tb.x0, y0 = tb.y0, z0 = tb.z0, z1 = tb.z1;
    const int tid = threadIdx.x;

    constexpr int PO = (TX * TY + NT - 1) / NT;
    static_assert(PO <= 32, "output mask is 32 bits");
    int oglb[PO];
    unsigned omask = 0;
#pragma unroll
    for (int i = 0; i < PO; ++i) {
        const int p = tid + NT * i;
        const int ty = p / TX, tx = p % TX;
        const bool ok = p < TX * TY && x0 + tx <= g.nx && y0 + ty <= g.ny;
        oglb[i] = ok ? (int)((y0 + ty) * g.sy + x0 + tx) : 0;
        omask |= ok ? 1u << i : 0u;
    }
    auto write_rows = [&](const T* lo, T* dp) {
#pragma unroll
        for (int i = 0; i < PO; ++i)
            if ((omask >> i) & 1u) st_stream(dp + oglb[i], lo[tid + NT * i]);
    };

    int off[M];   // y*sy + x of the column (32-bit: checked on the host)
    int flags[M]; // bit0 valid, bit1 interior in T+1, bit2 interior in T, bit3 colour parity
    int oidx[M];  // index of the column in the tile T (row-major), for the output rows
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int c = tid + NT * m;
        const int ly = c / W, lx = c % W;
        const int64_t x = x0 - 2 + lx, y = y0 - 2 + ly;
        const bool valid = c < NCOL && x >= 0 && x <= g.nx + 1 && y >= 0 && y <= g.ny + 1;
        const bool interior = valid && x >= 1 && x <= g.nx && y >= 1 && y <= g.ny;
        const bool t1 = interior && lx >= 1 && lx <= TX + 2 && ly >= 1 && ly <= TY + 2;
        const bool t0 = interior && lx >= 2 && lx <= TX + 1 && ly >= 2 && ly <= TY + 1;
        const int par = (int)(((x - 1) + (y - 1) + g.parity) & 1);
        flags[m] = (valid ? 1 : 0) | (t1 ? 2 : 0) | (t0 ? 4 : 0) | (par << 3);
        off[m] = valid ? (int)(y * g.sy + x) : 0;
        oidx[m] = (ly - 2) * TX + (lx - 2);
    }

    // register rings: the slot of plane p is (p - z0 + 3) mod R for u and b
    T U[R][M];
    T B[R][M];
    auto load_u = [&](int64_t k, T* v) {
        const bool kin = k >= 0 && k <= g.nz + 1;
        const T* sp = src + (kin ? k : 0) * g.sz;
#pragma unroll
        for (int m = 0; m < M; ++m) v[m] = (kin && (flags[m] & 1)) ? sp[off[m]] : T(0);
    };
    auto load_b = [&](int64_t k, T* v) {
        const bool kin = k >= 1 && k <= g.nz;
        const T* bp = b + (kin ? k : 0) * g.sz;
#pragma unroll
        for (int m = 0; m < M; ++m) v[m] = (kin && (flags[m] & 2)) ? bp[off[m]] : T(0);
    };
#pragma unroll
    for (int m = 0; m < M; ++m) {
        U[0][m] = T(0);
        B[1][m] = T(0);
    }
#pragma unroll
    for (int d = 0; d < D + 2; ++d) load_u(z0 - 2 + d, U[1 + d]);  // planes z0-2 .. z0-1+D
#pragma unroll
    for (int d = 0; d < D; ++d) load_b(z0 - 1 + d, B[2 + d]);      // b of z0-1 .. z0-2+D

    for (int64_t kb = z0 - 1; kb <= z1; kb += R) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t k = kb + r;
            if (k > z1) break;
            T* u_km2 = U[r % R];
            T* u_km1 = U[(r + 1) % R];
            T* u_k = U[(r + 2) % R];
            T* u_kp1 = U[(r + 3) % R];
            T* b_km1 = B[(r + 1) % R];
            T* b_k = B[(r + 2) % R];
            // prefetch plane k+1+D and b of plane k+D (used D steps later)
            if (k + 1 + D <= z1 + 1) load_u(k + 1 + D, U[(r + 3 + D) % R]);
            if (k + D <= z1) load_b(k + D, B[(r + 2 + D) % R]);
            T* lk = lds[k & 1][0];
            T* lkm1 = lds[k & 1][1];
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const int c = tid + NT * m;
                if (c < NCOL) {
                    lk[c] = u_k[m];
                    lkm1[c] = u_km1[m];
                }
            }
            __syncthreads();
            // plane k-2, finished at step k-1
            if (k - 2 >= z0 && k - 2 < z1) write_rows(lout[(k - 1) & 1], dst + (k - 2) * g.sz);
            const bool do_red = k >= 1 && k <= g.nz;
            const bool do_black = k - 1 >= z0 && k - 1 < z1;
            const int kc = (int)((k - 1) & 1);
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const int c = tid + NT * m;
                const bool sel = (((flags[m] >> 3) + kc) & 1) == 0;
                if (do_red && (flags[m] & 2) && sel) {
                    const T zm = u_km1[m], zp = u_kp1[m];
                    auto ld = [&](int ox, int oy, int oz) -> T {
                        return oz < 0 ? zm : oz > 0 ? zp : lk[c + oy * W + ox];
                    };
                    u_k[m] = gs_value<T, 3, FD>(h2, b_k[m], ld);
                }
            }
            T* lo = lout[k & 1];
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const int c = tid + NT * m;
                const bool sel = (((flags[m] >> 3) + kc) & 1) == 0;
                // (x, y, k-1) is black exactly when (x, y, k) is red
                if (do_black && (flags[m] & 4) && sel) {
                    const T zm = u_km2[m], zp = u_k[m];
                    auto ld = [&](int ox, int oy, int oz) -> T {
                        return oz < 0 ? zm : oz > 0 ? zp : lkm1[c + oy * W + ox];
                    };
                    u_km1[m] = gs_value<T, 3, FD>(h2, b_km1[m], ld);
                }
                if (do_black && (flags[m] & 4)) lo[oidx[m]] = u_km1[m];
            }
        }
    }
    // the last plane, z1 - 1, was finished at step z1
    __syncthreads();
    if (z1 - 1 >= z0) write_rows(lout[z1 & 1], dst + (z1 - 1) * g.sz);
}

// ---------------------------------------------------------------------------
// Two red-black sweeps of the 7-point stencil in one pass over memory.
//
// The second sweep trails the first by two planes.  At plane step k: the red
// points of plane k take their first-sweep values (from the previous
// iterate), the black points of plane k-1 theirs (from those reds), the red
// points of plane k-2 their second-sweep values (from the first-sweep
// blacks), and the black points of plane k-3 theirs; plane k-3 is then final.
// Every value is computed from the same neighbour values as in the four colour
// passes, so the result equals them bit for bit.  A tile recomputes the rings
// it needs -- first-sweep red on T+3, black on T+2, second-sweep red on T+1,
// black on T -- from the previous iterate on T+4.  A column (x, y) takes part
// in all four updates of a step or in none: (x, y, k) red means (x, y, k-1)
// black, (x, y, k-2) red, (x, y, k-3) black.
//
// Each thread owns columns of T+4 and keeps planes k-4 .. k+1+D of them, and
// their b values, in a register ring; the loop is unrolled over the ring, so
// no value is moved.  The in-plane neighbours come from LDS snapshots of planes
// k, k-1, k-2 and k-3 taken at the top of the step, when each holds what its
// update reads.  NB = 2 alternates two snapshot sets (one barrier per step),
// NB = 1 reuses one (two barriers).  The finished plane goes to an LDS row
// buffer and is stored by whole rows one step later.  A chunk of output planes
// [z0, z1) runs steps z0-3 .. z1+2 and reads u on planes z0-4 .. z1+3.
// ---------------------------------------------------------------------------
template <typename T, int TX, int TY, int NT, int D, int NB>
__device__ __forceinline__ void fd3_tile_two(const T* __restrict__ src, T* __restrict__ dst,
                                             const T* __restrict__ b, const Geo& g, T h2,
                                             const TileBox& tb)
{
    constexpr int W = TX + 8, HH = TY + 8, NCOL = W * HH;
    constexpr int M = (NCOL + NT - 1) / NT;
    constexpr int R = 6 + D;
    __shared__ T lds[NB][4][NCOL];
    __shared__ T lout[2][TX * TY];
    const int64_t x0 = tb.x0, y0 = tb.y0, z0 = tb.z0, z1 = tb.z1;
    const int tid = threadIdx.x;

    constexpr int PO = (TX * TY + NT - 1) / NT;
    static_assert(PO <= 32, "output mask is 32 bits");
    int oglb[PO];
    unsigned omask = 0;
#pragma unroll
    for (int i = 0; i < PO; ++i) {
        const int p = tid + NT * i;
        const int ty = p / TX, tx = p % TX;
        const bool ok = p < TX * TY && x0 + tx <= g.nx && y0 + ty <= g.ny;
        oglb[i] = ok ? (int)((y0 + ty) * g.sy + x0 + tx) : 0;
        omask |= ok ? 1u << i : 0u;
    }
    auto write_rows = [&](const T* lo, T* dp) {
#pragma unroll
        for (int i = 0; i < PO; ++i)
            if ((omask >> i) & 1u) st_stream(dp + oglb[i], lo[tid + NT * i]);
    };

    // flags: bit0 valid; bits 1..4 interior and inside T+3, T+2, T+1, T;
    // bit5 colour parity of (x, y)
    int off[M], flags[M], oidx[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int c = tid + NT * m;
        const int ly = c / W, lx = c % W;
        const int64_t x = x0 - 4 + lx, y = y0 - 4 + ly;
        const bool valid = c < NCOL && x >= 0 && x <= g.nx + 1 && y >= 0 && y <= g.ny + 1;
        const bool interior = valid && x >= 1 && x <= g.nx && y >= 1 && y <= g.ny;
        int f = valid ? 1 : 0;
#pragma unroll
        for (int r = 1; r <= 4; ++r) {
            const bool in = interior && lx >= r && lx <= W - 1 - r && ly >= r && ly <= HH - 1 - r;
            f |= in ? 1 << r : 0;
        }
        const int par = (int)(((x - 1) + (y - 1) + g.parity) & 1);
        flags[m] = f | (par << 5);
        off[m] = valid ? (int)(y * g.sy + x) : 0;
        oidx[m] = (ly - 4) * TX + (lx - 4);
    }

    T U[R][M];
    T B[R][M];
    auto load_u = [&](int64_t k, T* v) {
        const bool kin = k >= 0 && k <= g.nz + 1;
        const T* sp = src + (kin ? k : 0) * g.sz;
#pragma unroll
        for (int m = 0; m < M; ++m) v[m] = (kin && (flags[m] & 1)) ? sp[off[m]] : T(0);
    };
    auto load_b = [&](int64_t k, T* v) {
        const bool kin = k >= 1 && k <= g.nz;
        const T* bp = b + (kin ? k : 0) * g.sz;
#pragma unroll
        for (int m = 0; m < M; ++m) v[m] = (kin && (flags[m] & 2)) ? bp[off[m]] : T(0);
    };
    // plane p lives in ring slot (p - k0 + 4) mod R
    const int64_t k0 = z0 - 3, klast = z1 + 2;
#pragma unroll
    for (int s = 0; s < R; ++s)
#pragma unroll
        for (int m = 0; m < M; ++m) {
            U[s][m] = T(0);
            B[s][m] = T(0);
        }
#pragma unroll
    for (int d = 0; d < D + 2; ++d) load_u(k0 - 1 + d, U[3 + d]);  // planes k0-1 .. k0+D
#pragma unroll
    for (int d = 0; d < D; ++d) load_b(k0 + d, B[4 + d]);          // b of k0 .. k0+D-1

    // planes each update runs on (besides being interior planes)
    auto in_range = [&](int64_t p, int64_t lo, int64_t hi) { return p >= lo && p <= hi && p >= 1 && p <= g.nz; };
    for (int64_t kb = k0; kb <= klast; kb += R) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t k = kb + r;
            if (k > klast) break;
            T* u4 = U[r % R];        // plane k-4
            T* u3 = U[(r + 1) % R];  // k-3
            T* u2 = U[(r + 2) % R];  // k-2
            T* u1 = U[(r + 3) % R];  // k-1
            T* u0 = U[(r + 4) % R];  // k
            T* up = U[(r + 5) % R];  // k+1
            const T* b3 = B[(r + 1) % R];
            const T* b2 = B[(r + 2) % R];
            const T* b1 = B[(r + 3) % R];
            const T* b0 = B[(r + 4) % R];
            if (k + 1 + D <= z1 + 3) load_u(k + 1 + D, U[(r + 5 + D) % R]);
            if (k + D <= klast) load_b(k + D, B[(r + 4 + D) % R]);
            if (NB == 1) __syncthreads();
            T (*snap)[NCOL] = lds[NB == 2 ? (int)(k & 1) : 0];
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const int c = tid + NT * m;
                if (c < NCOL) {
                    snap[0][c] = u0[m];
                    snap[1][c] = u1[m];
                    snap[2][c] = u2[m];
                    snap[3][c] = u3[m];
                }
            }
            __syncthreads();
            // plane k-4, finished at step k-1
            if (k - 4 >= z0 && k - 4 < z1) write_rows(lout[(k - 1) & 1], dst + (k - 4) * g.sz);
            const bool r1 = in_range(k, z0 - 3, z1 + 2);
            const bool k1 = in_range(k - 1, z0 - 2, z1 + 1);
            const bool r2 = in_range(k - 2, z0 - 1, z1);
            const bool k2 = in_range(k - 3, z0, z1 - 1);
            const int kc = (int)((k - 1) & 1);
            T* lo = lout[k & 1];
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const int c = tid + NT * m;
                const int f = flags[m];
                const bool sel = (((f >> 5) + kc) & 1) == 0;  // (x, y, k) red
                if (sel) {
                    auto upd = [&](const T* pl, T zm, T zp, T bq) -> T {
                        auto ld = [&](int ox, int oy, int oz) -> T {
                            return oz < 0 ? zm : oz > 0 ? zp : pl[c + oy * W + ox];
                        };
                        return gs_value<T, 3, FD>(h2, bq, ld);
                    };
                    if (r1 && (f & 2)) u0[m] = upd(snap[0], u1[m], up[m], b0[m]);
                    if (k1 && (f & 4)) u1[m] = upd(snap[1], u2[m], u0[m], b1[m]);
                    if (r2 && (f & 8)) u2[m] = upd(snap[2], u3[m], u1[m], b2[m]);
                    if (k2 && (f & 16)) u3[m] = upd(snap[3], u4[m], u2[m], b3[m]);
                }
                if (k2 && (f & 16)) lo[oidx[m]] = u3[m];
            }
        }
    }
    // the last plane, z1 - 1, was finished at step z1 + 2
    __syncthreads();
    if (z1 - 1 >= z0) write_rows(lout[klast & 1], dst + (z1 - 1) * g.sz);
}

// ---------------------------------------------------------------------------
// 8-colour sweep of the 27-point trilinear stencil.
//
// Colour = px + 2 py + 4 pz (parities of x, y, z).  The face weights of this
// stencil are zero, so two colours that differ only in px never read each
// other: colours {0,1} (py = 0, pz = 0), {2,3}, {4,5}, {6,7} are four row
// phases A, B, C, D, each one a set of whole x-rows, and running a pair at
// once equals running its two colours one after the other.  A and B live on
// "even" planes (pz = 0), C and D on "odd" planes (pz = 1).  A reads only
// values of the previous iterate; B reads the new A rows of its plane; C and D
// read the final values of both neighbouring even planes, and D also the new C
// rows.  The sweep therefore streams through z in double steps: even plane e
// (A then B), then odd plane e-1 (C then D), after which planes e-1 and e are
// final.  A tile needs a recomputed halo of 4 (A on T+3, B on T+2, C on T+1,
// D on T).  Four planes (e-2 .. e+1) of the region T+4 live in LDS; the next
// two planes are prefetched into registers.  Neighbour sums keep the
// lexicographic offset order, so values equal the eight colour passes bit
// for bit.
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// The same 27-point sweep with two x-adjacent points per thread.  The finished
// planes leave through LDS: the tile's rows of planes e-1 and e, final after
// double step e, are stored during double step e+2 by whole wavefronts per row
// (full cache lines), instead of each pair storing its two points.  A fifth
// LDS slot keeps them until then.
//
// Points of one row phase are taken in pairs (x, x+1) whose left neighbour
// column x-1 is even in LDS, over the full width of T+3 in every phase (the
// extra ring points of the inner phases are computed but never used: they are
// written neither outside the interior nor to dst, and no point that is used
// reads them).  A pair reads 4 columns x-1..x+2 of the 8 neighbour rows,
// 32 values instead of 2 x 20, in 16-byte LDS loads; each point's sum is the
// same ordered fused multiply-add chain as the single-point form.
// ---------------------------------------------------------------------------
template <int TX, int TY, int NT, int HALO>
struct Q1Pairs {
    static constexpr int W = TX + 8;
    static constexpr int NPC = (TX + 6) / 2;             // pair columns across T+3
    static constexpr int ROWS = (TY + 2 * HALO + 1) / 2;  // rows of one type, at most
    static constexpr int P = (ROWS * NPC + NT - 1) / NT;  // pairs per thread, at most
};

// flags: bit0/bit1 left/right point interior, bit2/bit3 left/right inside T
template <int TX, int TY, int NT, int HALO, int P>
__device__ __forceinline__ void q1_make_pairs(const Geo& g, int64_t x0, int64_t y0, int rho,
                                              int* pc, int* poff, int* pfl)
{
    constexpr int W = TX + 8;
    constexpr int NPC = (TX + 6) / 2;
    const int ly_lo = 4 - HALO;
    const int rt_lo = (int)((y0 - 4 + ly_lo - 1 + g.parity) & 1);
    const int first = ly_lo + ((rho - rt_lo) & 1);
    const int nrows = (TY + 2 * HALO - (first - ly_lo) + 1) / 2;
#pragma unroll
    for (int i = 0; i < P; ++i) {
        const int sidx = (int)threadIdx.x + NT * i;
        const int row = sidx / NPC, pcol = sidx % NPC;
        const int ly = first + 2 * row, lx = 1 + 2 * pcol;
        const int64_t x = x0 - 4 + lx, y = y0 - 4 + ly;
        const bool rowok = row < nrows && y >= 1 && y <= g.ny;
        const bool in0 = rowok && x >= 1 && x <= g.nx;
        const bool in1 = rowok && x + 1 >= 1 && x + 1 <= g.nx;
        const bool ty_in = ly >= 4 && ly < 4 + TY;
        const bool out0 = in0 && ty_in && lx >= 4 && lx < 4 + TX;
        const bool out1 = in1 && ty_in && lx + 1 >= 4 && lx + 1 < 4 + TX;
        pc[i] = (in0 || in1) ? ly * W + lx : -1;
        poff[i] = (in0 || in1) ? (int)(y * g.sy + x) : 0;
        pfl[i] = (in0 ? 1 : 0) | (in1 ? 2 : 0) | (out0 ? 4 : 0) | (out1 ? 8 : 0);
    }
}

template <typename T, int P>
__device__ __forceinline__ void q1_load_b_pairs(const T* __restrict__ b, const Geo& g, int64_t k,
                                                const int* poff, const int* pfl, T* v)
{
    const bool kin = k >= 1 && k <= g.nz;
    const T* bp = b + (kin ? k : 0) * g.sz;
#pragma unroll
    for (int i = 0; i < P; ++i) {
        v[2 * i] = (kin && (pfl[i] & 1)) ? bp[poff[i]] : T(0);
        v[2 * i + 1] = (kin && (pfl[i] & 2)) ? bp[poff[i] + 1] : T(0);
    }
}

template <typename T, int W, int P, bool ROWWISE>
__device__ __forceinline__ void q1_phase_pairs(bool active, const int* pc, const T* bv,
                                               const T* lm, T* lk, const T* lp, const int* pfl,
                                               T h2, int maxring = 1 << 20)
{
    // The two points of a pair form the lanes of a 2-vector: the terms with
    // ox = -1 and ox = +1 are the aligned column pairs (x-1, x) and (x+1, x+2)
    // as loaded, the ox = 0 term is (x, x+1).  Each lane runs the ordered
    // fused multiply-add chain of gs_value (same offsets, same weights), so
    // both points round exactly as the single-point form.  ROWWISE adds each
    // row's terms as soon as the row is loaded (the same order), which needs
    // far fewer registers than loading all eight rows first.
    typedef T v2 __attribute__((ext_vector_type(2)));
    if (!active) return;
#pragma unroll
    for (int i = 0; i < P; ++i) {
        const int c = pc[i];
        if (c < 0 || (pfl[i] >> 2) > maxring) continue;
        v2 acc = {T(0), T(0)};
        if (ROWWISE) {
#pragma unroll
            for (int oz = -1; oz <= 1; ++oz) {
                const T* pl = oz < 0 ? lm : (oz > 0 ? lp : lk);
#pragma unroll
                for (int oy = -1; oy <= 1; ++oy) {
                    if (oz == 0 && oy == 0) continue;  // faces zero, centre excluded
                    const v2* row = reinterpret_cast<const v2*>(pl + (c - 1 + oy * W));
                    const v2 a = row[0], bb = row[1];
#pragma unroll
                    for (int ox = -1; ox <= 1; ++ox) {
                        const T w = weight<T, 3, Q1>(ox, oy, oz);
                        if (w == T(0)) continue;
                        const v2 val = ox < 0 ? a : (ox > 0 ? bb : (v2){a.y, bb.x});
                        const v2 wv = {w, w};
                        acc = __builtin_elementwise_fma(wv, val, acc);
                    }
                }
            }
        } else {
        v2 lo[3][3], hi[3][3];  // columns (x-1, x) and (x+1, x+2) of each row
#pragma unroll
        for (int oz = -1; oz <= 1; ++oz) {
            const T* pl = oz < 0 ? lm : (oz > 0 ? lp : lk);
#pragma unroll
            for (int oy = -1; oy <= 1; ++oy) {
                if (oz == 0 && oy == 0) continue;
                // c - 1 and W are even: 16-byte aligned for FP64
                const v2* row = reinterpret_cast<const v2*>(pl + (c - 1 + oy * W));
                lo[oz + 1][oy + 1] = row[0];
                hi[oz + 1][oy + 1] = row[1];
            }
        }
#pragma unroll
        for (int oz = -1; oz <= 1; ++oz)
#pragma unroll
            for (int oy = -1; oy <= 1; ++oy)
#pragma unroll
                for (int ox = -1; ox <= 1; ++ox) {
                    if (ox == 0 && oy == 0 && oz == 0) continue;
                    const T w = weight<T, 3, Q1>(ox, oy, oz);
                    if (w == T(0)) continue;
                    const v2 a = lo[oz + 1][oy + 1], bb = hi[oz + 1][oy + 1];
                    const v2 val = ox < 0 ? a : (ox > 0 ? bb : (v2){a.y, bb.x});
                    const v2 wv = {w, w};
                    acc = __builtin_elementwise_fma(wv, val, acc);
                }
        }
        const v2 bq = {bv[2 * i], bv[2 * i + 1]};
        const v2 h2v = {h2, h2};
        const v2 x = h2v * bq - acc;
        const T a0 = over_centre<T, 3, Q1>(x.x);
        const T a1 = over_centre<T, 3, Q1>(x.y);
        const int fl = pfl[i];
        if (fl & 1) lk[c] = a0;
        if (fl & 2) lk[c + 1] = a1;
    }
}

// VEC: the planes are loaded two columns per load instruction.  The LDS
// region starts at x0 - 4, an odd grid column (tiles start at x0 = 1 + TX i),
// and is TX + 8 wide, so the column pairs (lx, lx + 1) with lx even are the
// grid pairs (x, x + 1) with x odd: for a layout whose odd columns are
// aligned to two elements (the library's aligned layout, x = 1 on an aligned
// boundary, even strides) each is one aligned two-element load and one aligned
// two-element LDS store.  A pair with a column in the halo'd row is loaded
// whole: (-1, 0) reads the element before the row, (nx + 1, nx + 2) the row's
// first padding element, both inside the allocation (the launch checks the
// first row's and the last row's).  Their column outside the halo lands in
// LDS columns that only discarded values read.
template <typename T, int TX, int TY, int NT, bool ROWWISE = false, bool VEC = false>
__device__ __forceinline__ void q1_3_tile_pairs(const T* __restrict__ src, T* __restrict__ dst,
                                                const T* __restrict__ b, const Geo& g, T h2,
                                                const TileBox& tb)
{
    static_assert(TX % 2 == 0, "pairs need an even tile width");
    typedef T v2 __attribute__((ext_vector_type(2)));
    using LV = typename std::conditional<VEC, v2, T>::type;
    constexpr int W = TX + 8, HH = TY + 8, NCOL = W * HH;
    constexpr int LW = VEC ? 2 : 1;                        // columns per load
    constexpr int M = (NCOL / LW + NT - 1) / NT;
    using PA = Q1Pairs<TX, TY, NT, 3>;
    using PB = Q1Pairs<TX, TY, NT, 2>;
    using PC = Q1Pairs<TX, TY, NT, 1>;
    using PD = Q1Pairs<TX, TY, NT, 0>;
    // five plane slots: the planes e-2 .. e+1 a double step reads, and the
    // finished planes e-1 and e of the previous double step, which are written
    // out from LDS while the next step already fills its own two slots
    constexpr int NS = 5;
    __shared__ __attribute__((aligned(16))) T L[NS][NCOL];
    const int64_t x0 = tb.x0, y0 = tb.y0, z0 = tb.z0, z1 = tb.z1;
    auto slot = [&](int64_t p) -> T* {
        const int k = (int)(p - z0 + 3 * NS) % NS;  // p >= z0 - 3
        return (T*)__builtin_assume_aligned(L[k], 16);
    };
    const int tid = threadIdx.x;
    const int par = g.parity;

    // output points of the tile, whole rows per wavefront: LDS index and
    // in-plane offset; bit i of omask marks a point inside the grid
    constexpr int PO = (TX * TY + NT - 1) / NT;
    static_assert(PO <= 32, "output mask is 32 bits");
    int olds[PO], oglb[PO];
    unsigned omask = 0;
#pragma unroll
    for (int i = 0; i < PO; ++i) {
        const int p = tid + NT * i;
        const int ty = p / TX, tx = p % TX;
        const bool ok = p < TX * TY && x0 + tx <= g.nx && y0 + ty <= g.ny;
        olds[i] = (4 + ty) * W + 4 + tx;
        oglb[i] = ok ? (int)((y0 + ty) * g.sy + x0 + tx) : 0;
        omask |= ok ? 1u << i : 0u;
    }
    auto write_plane = [&](const T* lp, T* dp) {
#pragma unroll
        for (int i = 0; i < PO; ++i)
            if ((omask >> i) & 1u) st_stream(dp + oglb[i], lp[olds[i]]);
    };

    constexpr int kNoLoad = INT32_MIN;
    int coff[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int c = tid + NT * m;
        const int ly = c / (W / LW), lx = LW * (c % (W / LW));
        const int64_t x = x0 - 4 + lx, y = y0 - 4 + ly;
        const bool ok = c < NCOL / LW && y >= 0 && y <= g.ny + 1 && x >= 1 - LW && x <= g.nx + 1;
        coff[m] = ok ? (int)(y * g.sy + x) : kNoLoad;
    }
    int ca[PA::P], oa[PA::P], fa[PA::P], cb[PB::P], ob[PB::P], fb[PB::P];
    int cc[PC::P], oc[PC::P], fc[PC::P], cd[PD::P], od[PD::P], fd[PD::P];
    q1_make_pairs<TX, TY, NT, 3, PA::P>(g, x0, y0, 0, ca, oa, fa);
    q1_make_pairs<TX, TY, NT, 2, PB::P>(g, x0, y0, 1, cb, ob, fb);
    q1_make_pairs<TX, TY, NT, 1, PC::P>(g, x0, y0, 0, cc, oc, fc);
    q1_make_pairs<TX, TY, NT, 0, PD::P>(g, x0, y0, 1, cd, od, fd);

    auto is_even = [&](int64_t k) { return ((k - 1 + par) & 1) == 0; };
    const int64_t e_first = is_even(z0 - 1) ? z0 - 1 : z0;
    const int64_t e_last = is_even(z1) ? z1 : z1 - 1;

    auto load_plane = [&](int64_t k, LV* v) {
        const bool kin = k >= 0 && k <= g.nz + 1;
        const T* sp = src + (kin ? k : 0) * g.sz;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const bool ld = kin && coff[m] != kNoLoad;
            if constexpr (VEC)
                v[m] = ld ? *reinterpret_cast<const v2*>(sp + coff[m]) : v2{T(0), T(0)};
            else
                v[m] = ld ? sp[coff[m]] : T(0);
        }
    };
    auto store_plane = [&](const LV* v, T* lp) {
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int c = tid + NT * m;
            if (c < NCOL / LW) reinterpret_cast<LV*>(lp)[c] = v[m];
        }
    };

    LV n0[M], n1[M];
    T ba[2 * PA::P], bb[2 * PB::P], bc[2 * PC::P], bd[2 * PD::P];
    {
        LV t[M];
        load_plane(e_first - 1, t);
        store_plane(t, slot(e_first - 1));
    }
    load_plane(e_first, n0);
    load_plane(e_first + 1, n1);
    q1_load_b_pairs<T, PA::P>(b, g, e_first, oa, fa, ba);
    q1_load_b_pairs<T, PB::P>(b, g, e_first, ob, fb, bb);
    q1_load_b_pairs<T, PC::P>(b, g, e_first - 1, oc, fc, bc);
    q1_load_b_pairs<T, PD::P>(b, g, e_first - 1, od, fd, bd);

    // One double step e with the b values of this step in cb* and the next
    // step's loaded into nb*; the loop alternates the two register sets, so
    // no prefetched value is copied (a copy would wait for its load).
    T ba2[2 * PA::P], bb2[2 * PB::P], bc2[2 * PC::P], bd2[2 * PD::P];
    // planes finished by the previous double step, written out during the
    // next one (after its first barrier) so that the stores have a whole step
    // to drain before the next wait on the prefetched loads
    int64_t pend_e = -1, pend_o = -1;
    auto step = [&](int64_t e, const T* cba, const T* cbb, const T* cbc, const T* cbd, T* nba,
                    T* nbb, T* nbc, T* nbd) {
        T* lm2 = slot(e - 2);
        T* lm1 = slot(e - 1);
        T* l0 = slot(e);
        T* lp1 = slot(e + 1);
        store_plane(n0, l0);
        store_plane(n1, lp1);
        if (e + 2 <= e_last) {
            load_plane(e + 2, n0);
            load_plane(e + 3, n1);
            q1_load_b_pairs<T, PA::P>(b, g, e + 2, oa, fa, nba);
            q1_load_b_pairs<T, PB::P>(b, g, e + 2, ob, fb, nbb);
            q1_load_b_pairs<T, PC::P>(b, g, e + 1, oc, fc, nbc);
            q1_load_b_pairs<T, PD::P>(b, g, e + 1, od, fd, nbd);
        }
        __syncthreads();
        if (pend_e >= 0) write_plane(slot(pend_e), dst + pend_e * g.sz);
        if (pend_o >= 0) write_plane(slot(pend_o), dst + pend_o * g.sz);
        const bool ab = e >= 1 && e <= g.nz;
        q1_phase_pairs<T, W, PA::P, ROWWISE>(ab, ca, cba, lm1, l0, lp1, fa, h2);
        __syncthreads();
        q1_phase_pairs<T, W, PB::P, ROWWISE>(ab, cb, cbb, lm1, l0, lp1, fb, h2);
        __syncthreads();
        const int64_t o = e - 1;
        const bool cdo = o >= z0 && o < z1 && o >= 1 && o <= g.nz;
        q1_phase_pairs<T, W, PC::P, ROWWISE>(cdo, cc, cbc, lm2, lm1, l0, fc, h2);
        __syncthreads();
        q1_phase_pairs<T, W, PD::P, ROWWISE>(cdo, cd, cbd, lm2, lm1, l0, fd, h2);
        __syncthreads();
        // planes e (rows A, B) and e-1 (rows C, D) are final; their slots are
        // not refilled before the top of double step e+4
        pend_e = (ab && e >= z0 && e < z1) ? e : -1;
        pend_o = cdo ? o : -1;
    };
    for (int64_t e = e_first; e <= e_last; e += 4) {
        step(e, ba, bb, bc, bd, ba2, bb2, bc2, bd2);
        if (e + 2 > e_last) break;
        step(e + 2, ba2, bb2, bc2, bd2, ba, bb, bc, bd);
    }
    if (pend_e >= 0) write_plane(slot(pend_e), dst + pend_e * g.sz);
    if (pend_o >= 0) write_plane(slot(pend_o), dst + pend_o * g.sz);
}

// ---------------------------------------------------------------------------
// Two 8-colour sweeps of the 27-point stencil per pass over memory.
//
// The second sweep trails the first: at double step e (e an even plane) the
// eight row phases run in the order of the colour passes,
//     A1(e) B1(e) C1(e-1) D1(e-1)  A2(e-2) B2(e-2) C2(e-3) D2(e-3)
// (A..D as in the one-sweep body, 1 and 2 the sweep).  A2(e-2) reads the
// first-sweep values of planes e-3..e-1, all final after D1(e-1); C2(e-3)
// reads the second-sweep A and B rows of planes e-4 and e-2 and the first-
// sweep D rows of its own plane, which D2 overwrites only after.  So each
// update reads exactly the values of the sixteen colour passes, and planes e-3
// and e-2 are final after the step.  The values are updated in place in the
// LDS plane slots: a first-sweep value is last read before the second-sweep
// phase of its plane overwrites it.
//
// Neighbouring tiles run independently, so the first sweep is recomputed on a
// ring of 7 points around the tile T (A1 on T+7 down to D1 on T+4) and the
// second on T+3 .. T; u is loaded on T+8.  A pair list per row type serves
// both sweeps (the second-sweep phase skips the pairs of rows outside its
// ring), so a point is updated by the same thread in both sweeps and its
// right-hand side is loaded once per pass and kept in registers for two
// steps.  Along x every phase covers the full width of T+7; values computed on
// an x ring beyond the phase's own are never read by a value that is used.
// Along z a chunk [z0, z1) computes first-sweep rows on the planes z0-3 ..
// z1+2 and second-sweep rows on z0-1 .. z1, so its own planes are exact.
// Seven plane slots: the six planes e-4 .. e+1 a step reads and one more, so
// the finished planes e-3 and e-2 are stored by whole rows during the next
// step.
// ---------------------------------------------------------------------------
template <int TX, int TY, int NT, int RING>
struct Q1Pairs2 {
    static constexpr int NPC = (TX + 14) / 2;             // pair columns across T+7
    static constexpr int ROWS = (TY + 2 * RING + 1) / 2;  // rows of one type, at most
    static constexpr int P = (ROWS * NPC + NT - 1) / NT;  // pairs per thread, at most
};

// Pairs of one row type rho on the rows of T+RING and the columns of T+7:
// LDS index of the left point (region T+8, x0 - 8 at column 0), in-plane
// offset, and flags: bit0/bit1 left/right point interior, bits 2.. the row's
// ring (its distance from T along y).
template <int TX, int TY, int NT, int RING, int P>
__device__ __forceinline__ void q1_make_pairs2(const Geo& g, int64_t x0, int64_t y0, int rho,
                                               int* pc, int* poff, int* pfl)
{
    constexpr int H = 8, W = TX + 16, NPC = (TX + 14) / 2;
    const int ly_lo = H - RING;
    const int rt_lo = (int)((y0 - H + ly_lo - 1 + g.parity) & 1);
    const int first = ly_lo + ((rho - rt_lo) & 1);
    const int nrows = (TY + 2 * RING - (first - ly_lo) + 1) / 2;
#pragma unroll
    for (int i = 0; i < P; ++i) {
        const int sidx = (int)threadIdx.x + NT * i;
        const int row = sidx / NPC, pcol = sidx % NPC;
        const int ly = first + 2 * row, lx = 1 + 2 * pcol;
        const int64_t x = x0 - H + lx, y = y0 - H + ly;
        const bool rowok = row < nrows && y >= 1 && y <= g.ny;
        const bool in0 = rowok && x >= 1 && x <= g.nx;
        const bool in1 = rowok && x + 1 >= 1 && x + 1 <= g.nx;
        const int below = H - ly, above = ly - (H + TY - 1);
        const int ring = below > 0 ? below : (above > 0 ? above : 0);
        pc[i] = (in0 || in1) ? ly * W + lx : -1;
        poff[i] = (in0 || in1) ? (int)(y * g.sy + x) : 0;
        pfl[i] = (in0 ? 1 : 0) | (in1 ? 2 : 0) | (ring << 2);
    }
}

template <typename T, int TX, int TY, int NT>
__device__ __forceinline__ void q1_3_tile_two(const T* __restrict__ src, T* __restrict__ dst,
                                              const T* __restrict__ b, const Geo& g, T h2,
                                              const TileBox& tb)
{
    static_assert(TX % 2 == 0, "pairs need an even tile width");
    constexpr int H = 8, W = TX + 16, HH = TY + 16, NCOL = W * HH;
    constexpr int M = (NCOL + NT - 1) / NT;
    using PA = Q1Pairs2<TX, TY, NT, 7>;
    using PB = Q1Pairs2<TX, TY, NT, 6>;
    using PC = Q1Pairs2<TX, TY, NT, 5>;
    using PD = Q1Pairs2<TX, TY, NT, 4>;
    constexpr int NS = 7;
    __shared__ __attribute__((aligned(16))) T L[NS][NCOL];
    const int64_t x0 = tb.x0, y0 = tb.y0, z0 = tb.z0, z1 = tb.z1;
    auto slot = [&](int64_t p) -> T* {
        const int k = (int)(p - z0 + 2 * NS) % NS;  // p >= z0 - 8
        return (T*)__builtin_assume_aligned(L[k], 16);
    };
    const int tid = threadIdx.x;
    const int par = g.parity;

    // output points of the tile, whole rows per wavefront
    constexpr int PO = (TX * TY + NT - 1) / NT;
    static_assert(PO <= 32, "output mask is 32 bits");
    int olds[PO], oglb[PO];
    unsigned omask = 0;
#pragma unroll
    for (int i = 0; i < PO; ++i) {
        const int p = tid + NT * i;
        const int ty = p / TX, tx = p % TX;
        const bool ok = p < TX * TY && x0 + tx <= g.nx && y0 + ty <= g.ny;
        olds[i] = (H + ty) * W + H + tx;
        oglb[i] = ok ? (int)((y0 + ty) * g.sy + x0 + tx) : 0;
        omask |= ok ? 1u << i : 0u;
    }
    auto write_plane = [&](const T* lp, T* dp) {
#pragma unroll
        for (int i = 0; i < PO; ++i)
            if ((omask >> i) & 1u) st_stream(dp + oglb[i], lp[olds[i]]);
    };

    int coff[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int c = tid + NT * m;
        const int ly = c / W, lx = c % W;
        const int64_t x = x0 - H + lx, y = y0 - H + ly;
        const bool ok = c < NCOL && x >= 0 && x <= g.nx + 1 && y >= 0 && y <= g.ny + 1;
        coff[m] = ok ? (int)(y * g.sy + x) : -1;
    }
    int ca[PA::P], oa[PA::P], fa[PA::P], cb[PB::P], ob[PB::P], fb[PB::P];
    int cc[PC::P], oc[PC::P], fc[PC::P], cd[PD::P], od[PD::P], fd[PD::P];
    q1_make_pairs2<TX, TY, NT, 7, PA::P>(g, x0, y0, 0, ca, oa, fa);
    q1_make_pairs2<TX, TY, NT, 6, PB::P>(g, x0, y0, 1, cb, ob, fb);
    q1_make_pairs2<TX, TY, NT, 5, PC::P>(g, x0, y0, 0, cc, oc, fc);
    q1_make_pairs2<TX, TY, NT, 4, PD::P>(g, x0, y0, 1, cd, od, fd);

    auto is_even = [&](int64_t k) { return ((k - 1 + par) & 1) == 0; };
    // planes on which each sweep's rows are needed (see above)
    auto in1 = [&](int64_t p, int64_t lo, int64_t hi) {
        return p >= lo && p <= hi && p >= 1 && p <= g.nz;
    };
    const int64_t e_first = is_even(z0 - 3) ? z0 - 3 : z0 - 2;
    const int64_t e_last = is_even(z1 - 1) ? z1 + 1 : z1 + 2;

    auto load_plane = [&](int64_t k, T* v) {
        const bool kin = k >= 0 && k <= g.nz + 1;
        const T* sp = src + (kin ? k : 0) * g.sz;
#pragma unroll
        for (int m = 0; m < M; ++m) v[m] = (kin && coff[m] >= 0) ? sp[coff[m]] : T(0);
    };
    auto store_plane = [&](const T* v, T* lp) {
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int c = tid + NT * m;
            if (c < NCOL) lp[c] = v[m];
        }
    };

    // b of each row type for three double steps: the first sweep of this step
    // (cur), the second sweep of this step (old, loaded two steps ago) and the
    // next step (nxt, in flight); the loop rotates the three register sets.
    T ba0[2 * PA::P], ba1[2 * PA::P], ba2[2 * PA::P];
    T bb0[2 * PB::P], bb1[2 * PB::P], bb2[2 * PB::P];
    T bc0[2 * PC::P], bc1[2 * PC::P], bc2[2 * PC::P];
    T bd0[2 * PD::P], bd1[2 * PD::P], bd2[2 * PD::P];
    T n0[M], n1[M];
    {
        T t[M];
        for (int64_t p = e_first - 4; p < e_first; ++p) {
            load_plane(p, t);
            store_plane(t, slot(p));
        }
    }
    load_plane(e_first, n0);
    load_plane(e_first + 1, n1);
    // set 0: the first step's first sweep
    q1_load_b_pairs<T, PA::P>(b, g, e_first, oa, fa, ba0);
    q1_load_b_pairs<T, PB::P>(b, g, e_first, ob, fb, bb0);
    q1_load_b_pairs<T, PC::P>(b, g, e_first - 1, oc, fc, bc0);
    q1_load_b_pairs<T, PD::P>(b, g, e_first - 1, od, fd, bd0);
    // the second sweep starts two steps later (its first planes, e_first - 2
    // and e_first - 3, lie below z0 - 1): nothing to load for it yet
#pragma unroll
    for (int i = 0; i < 2 * PA::P; ++i) ba2[i] = T(0);
#pragma unroll
    for (int i = 0; i < 2 * PB::P; ++i) bb2[i] = T(0);
#pragma unroll
    for (int i = 0; i < 2 * PC::P; ++i) bc2[i] = T(0);
#pragma unroll
    for (int i = 0; i < 2 * PD::P; ++i) bd2[i] = T(0);

    int64_t pend_e = -1, pend_o = -1;
    auto step = [&](int64_t e, const T* cA, const T* cB, const T* cC, const T* cD, const T* oA,
                    const T* oB, const T* oC, const T* oD, T* nA, T* nB, T* nC, T* nD) {
        store_plane(n0, slot(e));
        store_plane(n1, slot(e + 1));
        if (e + 2 <= e_last) {
            load_plane(e + 2, n0);
            load_plane(e + 3, n1);
            q1_load_b_pairs<T, PA::P>(b, g, e + 2, oa, fa, nA);
            q1_load_b_pairs<T, PB::P>(b, g, e + 2, ob, fb, nB);
            q1_load_b_pairs<T, PC::P>(b, g, e + 1, oc, fc, nC);
            q1_load_b_pairs<T, PD::P>(b, g, e + 1, od, fd, nD);
        }
        __syncthreads();
        if (pend_e >= 0) write_plane(slot(pend_e), dst + pend_e * g.sz);
        if (pend_o >= 0) write_plane(slot(pend_o), dst + pend_o * g.sz);
        // first sweep: A, B on plane e; C, D on plane e-1
        const bool ab1 = in1(e, z0 - 3, z1 + 2);
        q1_phase_pairs<T, W, PA::P, true>(ab1, ca, cA, slot(e - 1), slot(e), slot(e + 1), fa, h2);
        __syncthreads();
        q1_phase_pairs<T, W, PB::P, true>(ab1, cb, cB, slot(e - 1), slot(e), slot(e + 1), fb, h2);
        __syncthreads();
        const bool cd1 = in1(e - 1, z0 - 2, z1 + 1);
        q1_phase_pairs<T, W, PC::P, true>(cd1, cc, cC, slot(e - 2), slot(e - 1), slot(e), fc, h2);
        __syncthreads();
        q1_phase_pairs<T, W, PD::P, true>(cd1, cd, cD, slot(e - 2), slot(e - 1), slot(e), fd, h2);
        __syncthreads();
        // second sweep: A, B on plane e-2; C, D on plane e-3
        const bool ab2 = in1(e - 2, z0 - 1, z1);
        q1_phase_pairs<T, W, PA::P, true>(ab2, ca, oA, slot(e - 3), slot(e - 2), slot(e - 1), fa, h2, 3);
        __syncthreads();
        q1_phase_pairs<T, W, PB::P, true>(ab2, cb, oB, slot(e - 3), slot(e - 2), slot(e - 1), fb, h2, 2);
        __syncthreads();
        const bool cd2 = in1(e - 3, z0, z1 - 1);
        q1_phase_pairs<T, W, PC::P, true>(cd2, cc, oC, slot(e - 4), slot(e - 3), slot(e - 2), fc, h2, 1);
        __syncthreads();
        q1_phase_pairs<T, W, PD::P, true>(cd2, cd, oD, slot(e - 4), slot(e - 3), slot(e - 2), fd, h2, 0);
        __syncthreads();
        // planes e-2 (A, B rows) and e-3 (C, D rows) are final; their slots
        // are refilled at the top of double steps e+4 and e+2 respectively,
        // after the write at the next step
        pend_e = (e - 2 >= z0 && e - 2 < z1 && e - 2 >= 1 && e - 2 <= g.nz) ? e - 2 : -1;
        pend_o = (e - 3 >= z0 && e - 3 < z1 && e - 3 >= 1 && e - 3 <= g.nz) ? e - 3 : -1;
    };
    // register sets rotate (cur, old, nxt): (0, 2, 1) -> (1, 0, 2) -> (2, 1, 0)
    for (int64_t e = e_first; e <= e_last; e += 6) {
        step(e, ba0, bb0, bc0, bd0, ba2, bb2, bc2, bd2, ba1, bb1, bc1, bd1);
        if (e + 2 > e_last) break;
        step(e + 2, ba1, bb1, bc1, bd1, ba0, bb0, bc0, bd0, ba2, bb2, bc2, bd2);
        if (e + 4 > e_last) break;
        step(e + 4, ba2, bb2, bc2, bd2, ba1, bb1, bc1, bd1, ba0, bb0, bc0, bd0);
    }
    if (pend_e >= 0) write_plane(slot(pend_e), dst + pend_e * g.sz);
    if (pend_o >= 0) write_plane(slot(pend_o), dst + pend_o * g.sz);
}

}  // namespace cs
