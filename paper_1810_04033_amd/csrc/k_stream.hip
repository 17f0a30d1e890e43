// Streaming stencil application for the separate-output-array sweeps (Sec. 2:
// a separate output array gives a mat-vec): weighted Jacobi and the residual,
// 3D grids.
//
// Each workgroup owns an xy tile T of TX x TY points and a chunk of z planes;
// it streams through z keeping the planes k-1, k, k+1 of the region T+1 in a
// ring of five LDS slots (the next plane is prefetched into registers one
// step ahead and stored two slots ahead, so one barrier per plane suffices).
// Every output point reads its neighbours from LDS in the lexicographic
// offset order of the plain definition, so the values match the point-wise
// kernels bit for bit.  The residual accumulates sum r^2, max |r| and sum b^2
// per thread in a fixed order and folds them per block into the partials
// consumed by the fixed-order second stage.
#include "cs_device.h"
#include "cs_internal.h"

#include <stdint.h>
#include <type_traits>

namespace cs {

namespace {

constexpr int kXcds = 8;

__device__ inline int64_t xcd_block(int64_t nblocks)
{
    const int64_t b = blockIdx.x;
    const int64_t per = nblocks / kXcds;
    const int64_t rem = nblocks % kXcds;
    const int64_t xcd = b % kXcds;
    const int64_t slot = b / kXcds;
    const int64_t start = xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per;
    return start + slot;
}

struct StreamWork {
    int tiles_x, tiles_y;
    int chunks;
    int64_t nblocks;
};

enum { MODE_JACOBI = 0, MODE_RESIDUAL = 1, MODE_IR = 2 };

__device__ inline void block_fold3(double& a, double& m, double& c, double* sh, int nt)
{
    const int t = threadIdx.x;
    sh[t] = a;
    sh[nt + t] = m;
    sh[2 * nt + t] = c;
    __syncthreads();
    for (int w = nt / 2; w > 0; w >>= 1) {
        if (t < w) {
            sh[t] = sh[t] + sh[t + w];
            sh[nt + t] = fmax(sh[nt + t], sh[nt + t + w]);
            sh[2 * nt + t] = sh[2 * nt + t] + sh[2 * nt + t + w];
        }
        __syncthreads();
    }
    a = sh[0];
    m = sh[nt];
    c = sh[2 * nt];
}

// S: storage type; the arithmetic type is S for Jacobi and double for the
// residual.
// MODE_IR (S = double): the residual r = b - A x plus, at the same points of a
// second (FP32) layout g2, r32 = fl32(r * inv_scale) and e32 = 0.
template <typename S, int ST, int MODE, int TX, int TY, int NT>
__global__ void __launch_bounds__(NT)
k_stream3(const S* __restrict__ src, S* __restrict__ dst, const S* __restrict__ b, Geo g,
          double h2d, double omegad, StreamWork wk, Partial* __restrict__ partials,
          Geo g2, float* __restrict__ r32, float* __restrict__ e32)
{
    using A = typename std::conditional<MODE == MODE_JACOBI, S, double>::type;
    constexpr int W = TX + 2, HH = TY + 2, NCOL = W * HH;
    constexpr int M = (NCOL + NT - 1) / NT;   // load columns per thread
    constexpr int P = (TX * TY + NT - 1) / NT;  // output points per thread
    constexpr int R = 5;
    __shared__ S L[R][NCOL];

    const int64_t work = xcd_block(wk.nblocks);
    const int64_t tiles = (int64_t)wk.tiles_x * wk.tiles_y;
    const int64_t chunk = work / tiles;
    const int64_t tile = work % tiles;
    const int64_t x0 = 1 + (tile % wk.tiles_x) * TX;
    const int64_t y0 = 1 + (tile / wk.tiles_x) * TY;
    const int64_t z0 = 1 + (chunk * g.nz) / wk.chunks;
    const int64_t z1 = 1 + ((chunk + 1) * g.nz) / wk.chunks;  // output planes [z0, z1)
    const int tid = threadIdx.x;

    int coff[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int c = tid + NT * m;
        const int ly = c / W, lx = c % W;
        const int64_t x = x0 - 1 + lx, y = y0 - 1 + ly;
        const bool ok = c < NCOL && x >= 0 && x <= g.nx + 1 && y >= 0 && y <= g.ny + 1;
        coff[m] = ok ? (int)(y * g.sy + x) : -1;
    }
    int pc[P], poff[P], poff2[MODE == MODE_IR ? P : 1];
#pragma unroll
    for (int i = 0; i < P; ++i) {
        const int s = tid + NT * i;
        const int ty = s / TX, tx = s % TX;
        const int64_t x = x0 + tx, y = y0 + ty;
        const bool ok = s < TX * TY && x <= g.nx && y <= g.ny;
        pc[i] = ok ? (ty + 1) * W + (tx + 1) : -1;
        poff[i] = ok ? (int)(y * g.sy + x) : 0;
        if (MODE == MODE_IR) poff2[i] = ok ? (int)(y * g2.sy + x) : 0;
    }

    auto load_plane = [&](int64_t k, S* v) {
        const bool kin = k >= 0 && k <= g.nz + 1;
        const S* sp = src + (kin ? k : 0) * g.sz;
#pragma unroll
        for (int m = 0; m < M; ++m) v[m] = (kin && coff[m] >= 0) ? sp[coff[m]] : S(0);
    };
    auto store_plane = [&](const S* v, S* lp) {
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int c = tid + NT * m;
            if (c < NCOL) lp[c] = v[m];
        }
    };
    auto load_b = [&](int64_t k, S* v) {
        const bool kin = k >= 1 && k <= g.nz;
        const S* bp = b + (kin ? k : 0) * g.sz;
#pragma unroll
        for (int i = 0; i < P; ++i) v[i] = (kin && pc[i] >= 0) ? bp[poff[i]] : S(0);
    };
    auto slot = [&](int64_t k) { return (int)((k - z0 + 2 * R) % R); };

    S pre[M], bcur[P], bnxt[P];
    {
        S t[M];
        load_plane(z0 - 1, t);
        store_plane(t, L[slot(z0 - 1)]);
        load_plane(z0, t);
        store_plane(t, L[slot(z0)]);
    }
    load_plane(z0 + 1, pre);
    load_b(z0, bcur);

    const A h2 = (A)h2d, omega = (A)omegad;
    double s_r2 = 0.0, mx = 0.0, s_b2 = 0.0;
    for (int64_t k = z0; k < z1; ++k) {
        store_plane(pre, L[slot(k + 1)]);
        if (k + 2 <= z1) load_plane(k + 2, pre);
        if (k + 1 < z1) load_b(k + 1, bnxt);
        __syncthreads();
        const S* lm = L[slot(k - 1)];
        const S* l0 = L[slot(k)];
        const S* lp = L[slot(k + 1)];
        S* dp = dst + k * g.sz;
#pragma unroll
        for (int i = 0; i < P; ++i) {
            const int c = pc[i];
            if (c < 0) continue;
            auto ld = [&](int ox, int oy, int oz) -> A {
                const S* pl = oz < 0 ? lm : (oz > 0 ? lp : l0);
                return (A)pl[c + oy * W + ox];
            };
            if (MODE == MODE_JACOBI) {
                st_stream(dp + poff[i], (S)jacobi_value<A, 3, ST>(h2, omega, (A)bcur[i], (A)l0[c], ld));
            } else {
                const double su = ordered_sum<double, 3, ST, true>(ld);
                const double bq = (double)bcur[i];
                const double rq = bq - su / h2d;
                if (MODE == MODE_RESIDUAL && dst) dp[poff[i]] = (S)rq;
                if (MODE == MODE_IR) {
                    r32[k * g2.sz + poff2[i]] = (float)(rq * omegad);
                    e32[k * g2.sz + poff2[i]] = 0.0f;
                }
                s_r2 += rq * rq;
                s_b2 += bq * bq;
                mx = fmax(mx, fabs(rq));
            }
        }
#pragma unroll
        for (int i = 0; i < P; ++i) bcur[i] = bnxt[i];
    }
    if (MODE != MODE_JACOBI) {
        __shared__ double sh[3 * NT];
        __syncthreads();
        block_fold3(s_r2, mx, s_b2, sh, NT);
        if (tid == 0) {
            partials[blockIdx.x].sum_r2 = s_r2;
            partials[blockIdx.x].max_r = mx;
            partials[blockIdx.x].sum_b2 = s_b2;
        }
    }
}

// Weighted Jacobi with the 27-point stencil, two x-adjacent points per thread.
// The pair (x, x+1) reads columns x-1..x+2 of the nine neighbour rows as 16-byte
// LDS loads and runs the two ordered fused multiply-add chains as the lanes of
// a 2-vector (the ox = -1 and +1 terms are the loaded column pairs, the ox = 0
// term a lane shuffle), so each point rounds exactly as jacobi_value.  The
// pair is stored as one 16-byte nontemporal store when the row layout makes
// it aligned (the library's padded layout does), else as two.
template <typename S, int TX, int TY, int NT>
__global__ void __launch_bounds__(NT)
k_jacobi3_q1_pairs(const S* __restrict__ src, S* __restrict__ dst, const S* __restrict__ b, Geo g,
                   double h2d, double omegad, StreamWork wk)
{
    typedef S v2 __attribute__((ext_vector_type(2)));
    static_assert(TX % 2 == 0 && (TX / 2) * TY == NT, "one pair per thread");
    constexpr int W = TX + 2, HH = TY + 2, NCOL = W * HH;
    constexpr int M = (NCOL + NT - 1) / NT;
    constexpr int R = 5;
    __shared__ __attribute__((aligned(16))) S L[R][NCOL];

    const int64_t work = xcd_block(wk.nblocks);
    const int64_t tiles = (int64_t)wk.tiles_x * wk.tiles_y;
    const int64_t chunk = work / tiles;
    const int64_t tile = work % tiles;
    const int64_t x0 = 1 + (tile % wk.tiles_x) * TX;
    const int64_t y0 = 1 + (tile / wk.tiles_x) * TY;
    const int64_t z0 = 1 + (chunk * g.nz) / wk.chunks;
    const int64_t z1 = 1 + ((chunk + 1) * g.nz) / wk.chunks;
    const int tid = threadIdx.x;

    int coff[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int c = tid + NT * m;
        const int ly = c / W, lx = c % W;
        const int64_t x = x0 - 1 + lx, y = y0 - 1 + ly;
        const bool ok = c < NCOL && x >= 0 && x <= g.nx + 1 && y >= 0 && y <= g.ny + 1;
        coff[m] = ok ? (int)(y * g.sy + x) : -1;
    }
    // this thread's pair: points (x, x+1) of row y
    const int tx = 2 * (tid % (TX / 2)), ty = tid / (TX / 2);
    const int64_t x = x0 + tx, y = y0 + ty;
    const bool in0 = x <= g.nx && y <= g.ny, in1 = x + 1 <= g.nx && y <= g.ny;
    const int cl = (ty + 1) * W + tx;  // column x-1 of the pair's row: even
    const int poff = in0 ? (int)(y * g.sy + x) : 0;

    auto load_plane = [&](int64_t k, S* v) {
        const bool kin = k >= 0 && k <= g.nz + 1;
        const S* sp = src + (kin ? k : 0) * g.sz;
#pragma unroll
        for (int m = 0; m < M; ++m) v[m] = (kin && coff[m] >= 0) ? sp[coff[m]] : S(0);
    };
    auto store_plane = [&](const S* v, S* lp) {
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int c = tid + NT * m;
            if (c < NCOL) lp[c] = v[m];
        }
    };
    auto load_b = [&](int64_t k, v2& v) {
        const bool kin = k >= 1 && k <= g.nz;
        const S* bp = b + (kin ? k : 0) * g.sz;
        v.x = (kin && in0) ? bp[poff] : S(0);
        v.y = (kin && in1) ? bp[poff + 1] : S(0);
    };
    auto slot = [&](int64_t k) { return (int)((k - z0 + 2 * R) % R); };

    S pre[M];
    v2 bcur, bnxt;
    {
        S t[M];
        load_plane(z0 - 1, t);
        store_plane(t, L[slot(z0 - 1)]);
        load_plane(z0, t);
        store_plane(t, L[slot(z0)]);
    }
    load_plane(z0 + 1, pre);
    load_b(z0, bcur);

    const S h2 = (S)h2d, omega = (S)omegad;
    const v2 h2v = {h2, h2}, omv = {omega, omega};
    for (int64_t k = z0; k < z1; ++k) {
        store_plane(pre, L[slot(k + 1)]);
        if (k + 2 <= z1) load_plane(k + 2, pre);
        if (k + 1 < z1) load_b(k + 1, bnxt);
        __syncthreads();
        const S* pls[3] = {L[slot(k - 1)], L[slot(k)], L[slot(k + 1)]};
        v2 lo[3][3], hi[3][3];
#pragma unroll
        for (int oz = 0; oz < 3; ++oz)
#pragma unroll
            for (int oy = 0; oy < 3; ++oy) {
                const v2* row = reinterpret_cast<const v2*>(pls[oz] + cl + (oy - 1) * W);
                lo[oz][oy] = row[0];
                hi[oz][oy] = row[1];
            }
        v2 acc = {S(0), S(0)};
#pragma unroll
        for (int oz = -1; oz <= 1; ++oz)
#pragma unroll
            for (int oy = -1; oy <= 1; ++oy)
#pragma unroll
                for (int ox = -1; ox <= 1; ++ox) {
                    const S w = weight<S, 3, Q1>(ox, oy, oz);
                    if (w == S(0)) continue;
                    const v2 a = lo[oz + 1][oy + 1], c2 = hi[oz + 1][oy + 1];
                    const v2 val = ox < 0 ? a : (ox > 0 ? c2 : (v2){a.y, c2.x});
                    const v2 wv = {w, w};
                    acc = __builtin_elementwise_fma(wv, val, acc);
                }
        const v2 ctr = {lo[1][1].y, hi[1][1].x};  // u at (x, y, k), (x+1, y, k)
        const v2 q = h2v * bcur - acc;
        const v2 sc = {over_centre<S, 3, Q1>(q.x), over_centre<S, 3, Q1>(q.y)};
        const v2 out = __builtin_elementwise_fma(omv, sc, ctr);
        S* dp = dst + k * g.sz + poff;
        if (in0 && in1 && (((uintptr_t)dp & (2 * sizeof(S) - 1)) == 0)) {
            __builtin_nontemporal_store(out, reinterpret_cast<v2*>(dp));
        } else {
            if (in0) st_stream(dp, out.x);
            if (in1) st_stream(dp + 1, out.y);
        }
        bcur = bnxt;
    }
}

// Two weighted Jacobi sweeps with the 7-point stencil in one pass over memory.
// The first sweep's iterate u1 = J(u) is computed on the tile grown by one
// point in x and y and kept in a three-plane LDS ring; the second sweep
// u2 = J(u1) is computed on the tile from that ring and stored.  u1 never goes
// to HBM, so the pass moves the bytes of one sweep for the updates of two.
// Every value is the same expression as in the one-sweep kernel, so the pair
// of sweeps gives the iterate of two one-sweep passes bit for bit.  Grown-tile
// points on the boundary keep their Dirichlet value (the halo of the work array
// holds the same values).
//
// A thread computes u1 and u2 at the same tile points, so b is loaded once per
// point and kept in a three-plane register ring (the z loop is unrolled by
// three, so the ring rotates without register moves); the ring of grown-tile
// points around the tile is spread over all threads.  Step k of the z loop
// computes u1 on plane k, then u2 on plane k - 1; a chunk of output planes
// [z0, z1) reads u on planes z0 - 2 .. z1 + 1.  Two barriers per plane: after
// the u plane is stored, and after the u1 plane is written.
template <typename S, int TX, int TY, int NT>
__global__ void __launch_bounds__(NT)
k_jacobi3_fd_two(const S* __restrict__ src, S* __restrict__ dst, const S* __restrict__ b, Geo g,
                 double h2d, double omegad, StreamWork wk)
{
    constexpr int W = TX + 4, HH = TY + 4, NCOL = W * HH;  // u on the tile + 2
    constexpr int W1 = TX + 2, H1 = TY + 2, N1 = W1 * H1;  // u1 on the tile + 1
    constexpr int NR = 2 * W1 + 2 * (H1 - 2);              // u1 points outside the tile
    constexpr int M = (NCOL + NT - 1) / NT;
    constexpr int P = (TX * TY + NT - 1) / NT;
    constexpr int PR = (NR + NT - 1) / NT;
    __shared__ S L[3][NCOL];
    __shared__ S L1[3][N1];

    const int64_t work = xcd_block(wk.nblocks);
    const int64_t tiles = (int64_t)wk.tiles_x * wk.tiles_y;
    const int64_t chunk = work / tiles;
    const int64_t tile = work % tiles;
    const int64_t x0 = 1 + (tile % wk.tiles_x) * TX;
    const int64_t y0 = 1 + (tile / wk.tiles_x) * TY;
    const int64_t z0 = 1 + (chunk * g.nz) / wk.chunks;
    const int64_t z1 = 1 + ((chunk + 1) * g.nz) / wk.chunks;
    const int tid = threadIdx.x;

    int coff[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int c = tid + NT * m;
        const int64_t x = x0 - 2 + c % W, y = y0 - 2 + c / W;
        const bool ok = c < NCOL && x >= 0 && x <= g.nx + 1 && y >= 0 && y <= g.ny + 1;
        coff[m] = ok ? (int)(y * g.sy + x) : -1;
    }
    // kind of a u1 point: 2 interior (computed), 1 boundary (keeps u), 0 outside
    auto kind_of = [&](int64_t x, int64_t y) {
        if (x > g.nx + 1 || y > g.ny + 1) return 0;
        return (x >= 1 && x <= g.nx && y >= 1 && y <= g.ny) ? 2 : 1;
    };
    // tile points (u1 and u2)
    int tk[P], tu[P], t1[P], toff[P];
#pragma unroll
    for (int i = 0; i < P; ++i) {
        const int t = tid + NT * i;
        const int tx = t % TX, ty = t / TX;
        const int64_t x = x0 + tx, y = y0 + ty;
        tk[i] = t < TX * TY ? kind_of(x, y) : 0;
        tu[i] = (ty + 2) * W + (tx + 2);
        t1[i] = (ty + 1) * W1 + (tx + 1);
        toff[i] = tk[i] == 2 ? (int)(y * g.sy + x) : 0;
    }
    // ring points (u1 only): top row, bottom row, left column, right column
    int rk[PR], ru[PR], r1[PR], roff[PR];
#pragma unroll
    for (int j = 0; j < PR; ++j) {
        const int r = tid + NT * j;
        int lx, ly;
        if (r < W1) {
            lx = r; ly = 0;
        } else if (r < 2 * W1) {
            lx = r - W1; ly = H1 - 1;
        } else {
            const int q = r - 2 * W1;
            lx = q < H1 - 2 ? 0 : W1 - 1;
            ly = 1 + q % (H1 - 2);
        }
        const int64_t x = x0 - 1 + lx, y = y0 - 1 + ly;
        rk[j] = r < NR ? kind_of(x, y) : 0;
        ru[j] = (ly + 1) * W + (lx + 1);
        r1[j] = ly * W1 + lx;
        roff[j] = rk[j] == 2 ? (int)(y * g.sy + x) : 0;
    }

    auto load_plane = [&](int64_t k, S* v) {
        const bool kin = k >= 0 && k <= g.nz + 1;
        const S* sp = src + (kin ? k : 0) * g.sz;
#pragma unroll
        for (int m = 0; m < M; ++m) v[m] = (kin && coff[m] >= 0) ? sp[coff[m]] : S(0);
    };
    auto store_plane = [&](const S* v, S* lp) {
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int c = tid + NT * m;
            if (c < NCOL) lp[c] = v[m];
        }
    };
    auto load_b = [&](int64_t k, S* bt, S* br) {
        const bool kin = k >= 1 && k <= g.nz;
        const S* bp = b + (kin ? k : 0) * g.sz;
#pragma unroll
        for (int i = 0; i < P; ++i) bt[i] = (kin && tk[i] == 2) ? bp[toff[i]] : S(0);
#pragma unroll
        for (int j = 0; j < PR; ++j) br[j] = (kin && rk[j] == 2) ? bp[roff[j]] : S(0);
    };
    auto slot = [&](int64_t k) { return (int)((k - z0 + 6) % 3); };

    const S h2 = (S)h2d, omega = (S)omegad;
    auto u1_point = [&](bool kint, int kind, int cu, S bq, const S* lm, const S* l0,
                        const S* lp) -> S {
        if (!(kint && kind == 2)) return l0[cu];
        auto ld = [&](int ox, int oy, int oz) -> S {
            const S* pl = oz < 0 ? lm : (oz > 0 ? lp : l0);
            return pl[cu + oy * W + ox];
        };
        return jacobi_value<S, 3, FD>(h2, omega, bq, l0[cu], ld);
    };

    S pre[M];
    S B0[P], B1[P], B2[P], R0[PR], R1[PR], R2[PR];
    {
        S t[M];
        load_plane(z0 - 2, t);
        store_plane(t, L[slot(z0 - 2)]);
        load_plane(z0 - 1, t);
        store_plane(t, L[slot(z0 - 1)]);
    }
    load_plane(z0, pre);
    load_b(z0 - 1, B0, R0);

    // step k: u1 on plane k with b of plane k (bu, ru_), u2 on plane k - 1
    // with b of plane k - 1 (bp2); b of plane k + 1 is loaded into (bn, rn)
    auto step = [&](int64_t k, const S* bu, const S* bp2, S* bn, const S* rb, S* rn) {
        store_plane(pre, L[slot(k + 1)]);
        if (k + 2 <= z1 + 1) load_plane(k + 2, pre);
        if (k + 1 <= z1) load_b(k + 1, bn, rn);
        __syncthreads();
        {
            const S* lm = L[slot(k - 1)];
            const S* l0 = L[slot(k)];
            const S* lp = L[slot(k + 1)];
            S* o = L1[slot(k)];
            const bool kint = k >= 1 && k <= g.nz;
#pragma unroll
            for (int i = 0; i < P; ++i)
                if (tk[i] != 0) o[t1[i]] = u1_point(kint, tk[i], tu[i], bu[i], lm, l0, lp);
#pragma unroll
            for (int j = 0; j < PR; ++j)
                if (rk[j] != 0) o[r1[j]] = u1_point(kint, rk[j], ru[j], rb[j], lm, l0, lp);
        }
        __syncthreads();
        if (k - 1 >= z0) {
            const S* lm = L1[slot(k - 2)];
            const S* l0 = L1[slot(k - 1)];
            const S* lp = L1[slot(k)];
            S* dp = dst + (k - 1) * g.sz;
#pragma unroll
            for (int i = 0; i < P; ++i) {
                if (tk[i] != 2) continue;
                const int c = t1[i];
                auto ld = [&](int ox, int oy, int oz) -> S {
                    const S* pl = oz < 0 ? lm : (oz > 0 ? lp : l0);
                    return pl[c + oy * W1 + ox];
                };
                st_stream(dp + toff[i], jacobi_value<S, 3, FD>(h2, omega, bp2[i], l0[c], ld));
            }
        }
    };
    for (int64_t k = z0 - 1; k <= z1; k += 3) {
        step(k, B0, B2, B1, R0, R1);
        if (k + 1 > z1) break;
        step(k + 1, B1, B0, B2, R1, R2);
        if (k + 2 > z1) break;
        step(k + 2, B2, B1, B0, R2, R0);
    }
}

// The 27-point pair update of k_jacobi3_q1_pairs on LDS plane data: the pair
// whose row starts (column x-1) at index cl of planes pl[0..2] (row stride RW).
template <typename S, int RW, typename V2>
__device__ __forceinline__ V2 q1_jacobi_pair(const S* const* pls, int cl, V2 bq, V2 h2v, V2 omv)
{
    V2 lo[3][3], hi[3][3];
#pragma unroll
    for (int oz = 0; oz < 3; ++oz)
#pragma unroll
        for (int oy = 0; oy < 3; ++oy) {
            const V2* row = reinterpret_cast<const V2*>(pls[oz] + cl + (oy - 1) * RW);
            lo[oz][oy] = row[0];
            hi[oz][oy] = row[1];
        }
    V2 acc = {S(0), S(0)};
#pragma unroll
    for (int oz = -1; oz <= 1; ++oz)
#pragma unroll
        for (int oy = -1; oy <= 1; ++oy)
#pragma unroll
            for (int ox = -1; ox <= 1; ++ox) {
                const S w = weight<S, 3, Q1>(ox, oy, oz);
                if (w == S(0)) continue;
                const V2 a = lo[oz + 1][oy + 1], c2 = hi[oz + 1][oy + 1];
                const V2 val = ox < 0 ? a : (ox > 0 ? c2 : (V2){a.y, c2.x});
                const V2 wv = {w, w};
                acc = __builtin_elementwise_fma(wv, val, acc);
            }
    const V2 ctr = {lo[1][1].y, hi[1][1].x};
    const V2 q = h2v * bq - acc;
    const V2 sc = {over_centre<S, 3, Q1>(q.x), over_centre<S, 3, Q1>(q.y)};
    return __builtin_elementwise_fma(omv, sc, ctr);
}

// Two weighted Jacobi sweeps with the 27-point stencil in one pass over memory:
// the structure of k_jacobi3_fd_two (u1 on the tile grown by one, b loaded once
// per point into a register ring) with the pair update of k_jacobi3_q1_pairs
// at the tile points of both sweeps.  A thread's u1 pairs are its u2 pairs
// (x, x+1), x - x0 even; the u plane region starts at x0 - 3 and the u1 region
// at x0 - 1, so the 16-byte loads of both updates are aligned (the region rows
// have even lengths).  The grown-tile points around the tile take the
// single-point form, which rounds identically.
template <typename S, int TX, int TY, int NT>
__global__ void __launch_bounds__(NT)
k_jacobi3_q1_two(const S* __restrict__ src, S* __restrict__ dst, const S* __restrict__ b, Geo g,
                 double h2d, double omegad, StreamWork wk)
{
    typedef S v2 __attribute__((ext_vector_type(2)));
    static_assert(TX % 2 == 0, "pairs");
    constexpr int W = TX + 6, HH = TY + 4, NCOL = W * HH;  // u: x0-3 .., y0-2 ..
    constexpr int W1 = TX + 2, H1 = TY + 2, N1 = W1 * H1;  // u1: x0-1 .., y0-1 ..
    constexpr int NR = 2 * W1 + 2 * (H1 - 2);
    constexpr int NPT = TX / 2 * TY;
    constexpr int M = (NCOL + NT - 1) / NT;
    constexpr int P = (NPT + NT - 1) / NT;
    constexpr int PR = (NR + NT - 1) / NT;
    __shared__ __attribute__((aligned(16))) S L[3][NCOL];
    __shared__ __attribute__((aligned(16))) S L1[3][N1];

    const int64_t work = xcd_block(wk.nblocks);
    const int64_t tiles = (int64_t)wk.tiles_x * wk.tiles_y;
    const int64_t chunk = work / tiles;
    const int64_t tile = work % tiles;
    const int64_t x0 = 1 + (tile % wk.tiles_x) * TX;
    const int64_t y0 = 1 + (tile / wk.tiles_x) * TY;
    const int64_t z0 = 1 + (chunk * g.nz) / wk.chunks;
    const int64_t z1 = 1 + ((chunk + 1) * g.nz) / wk.chunks;
    const int tid = threadIdx.x;

    int coff[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int c = tid + NT * m;
        const int64_t x = x0 - 3 + c % W, y = y0 - 2 + c / W;
        const bool ok = c < NCOL && x >= 0 && x <= g.nx + 1 && y >= 0 && y <= g.ny + 1;
        coff[m] = ok ? (int)(y * g.sy + x) : -1;
    }
    auto kind_of = [&](int64_t x, int64_t y) {
        if (x > g.nx + 1 || y > g.ny + 1) return 0;
        return (x >= 1 && x <= g.nx && y >= 1 && y <= g.ny) ? 2 : 1;
    };
    // tile pairs: kinds of both points, u row index of column x-1 (centre
    // row), u1 index of column x-1 (centre row), global offset of x
    int ka[P], kb[P], cu[P], c1[P], toff[P];
#pragma unroll
    for (int i = 0; i < P; ++i) {
        const int t = tid + NT * i;
        const int tx = 2 * (t % (TX / 2)), ty = t / (TX / 2);
        const int64_t x = x0 + tx, y = y0 + ty;
        ka[i] = t < NPT ? kind_of(x, y) : 0;
        kb[i] = t < NPT ? kind_of(x + 1, y) : 0;
        cu[i] = (ty + 2) * W + tx + 2;
        c1[i] = (ty + 1) * W1 + tx;
        toff[i] = ka[i] == 2 ? (int)(y * g.sy + x) : 0;
    }
    int rk[PR], ru[PR], r1[PR], roff[PR];
#pragma unroll
    for (int j = 0; j < PR; ++j) {
        const int r = tid + NT * j;
        int lx, ly;
        if (r < W1) {
            lx = r; ly = 0;
        } else if (r < 2 * W1) {
            lx = r - W1; ly = H1 - 1;
        } else {
            const int q = r - 2 * W1;
            lx = q < H1 - 2 ? 0 : W1 - 1;
            ly = 1 + q % (H1 - 2);
        }
        const int64_t x = x0 - 1 + lx, y = y0 - 1 + ly;
        rk[j] = r < NR ? kind_of(x, y) : 0;
        ru[j] = (ly + 1) * W + (lx + 2);
        r1[j] = ly * W1 + lx;
        roff[j] = rk[j] == 2 ? (int)(y * g.sy + x) : 0;
    }

    auto load_plane = [&](int64_t k, S* v) {
        const bool kin = k >= 0 && k <= g.nz + 1;
        const S* sp = src + (kin ? k : 0) * g.sz;
#pragma unroll
        for (int m = 0; m < M; ++m) v[m] = (kin && coff[m] >= 0) ? sp[coff[m]] : S(0);
    };
    auto store_plane = [&](const S* v, S* lp) {
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int c = tid + NT * m;
            if (c < NCOL) lp[c] = v[m];
        }
    };
    auto load_b = [&](int64_t k, v2* bt, S* br) {
        const bool kin = k >= 1 && k <= g.nz;
        const S* bp = b + (kin ? k : 0) * g.sz;
#pragma unroll
        for (int i = 0; i < P; ++i) {
            bt[i].x = (kin && ka[i] == 2) ? bp[toff[i]] : S(0);
            bt[i].y = (kin && kb[i] == 2) ? bp[toff[i] + 1] : S(0);
        }
#pragma unroll
        for (int j = 0; j < PR; ++j) br[j] = (kin && rk[j] == 2) ? bp[roff[j]] : S(0);
    };
    auto slot = [&](int64_t k) { return (int)((k - z0 + 6) % 3); };

    const S h2 = (S)h2d, omega = (S)omegad;
    const v2 h2v = {h2, h2}, omv = {omega, omega};

    S pre[M];
    v2 B0[P], B1[P], B2[P];
    S R0[PR], R1[PR], R2[PR];
    {
        S t[M];
        load_plane(z0 - 2, t);
        store_plane(t, L[slot(z0 - 2)]);
        load_plane(z0 - 1, t);
        store_plane(t, L[slot(z0 - 1)]);
    }
    load_plane(z0, pre);
    load_b(z0 - 1, B0, R0);

    auto step = [&](int64_t k, const v2* bu, const v2* bp2, v2* bn, const S* rb, S* rn) {
        store_plane(pre, L[slot(k + 1)]);
        if (k + 2 <= z1 + 1) load_plane(k + 2, pre);
        if (k + 1 <= z1) load_b(k + 1, bn, rn);
        __syncthreads();
        {
            const S* pls[3] = {L[slot(k - 1)], L[slot(k)], L[slot(k + 1)]};
            S* o = L1[slot(k)];
            const bool kint = k >= 1 && k <= g.nz;
#pragma unroll
            for (int i = 0; i < P; ++i) {
                if (ka[i] == 0 && kb[i] == 0) continue;
                const v2 out = q1_jacobi_pair<S, W>(pls, cu[i], bu[i], h2v, omv);
                const S* l0 = pls[1];
                o[c1[i] + 1] = (kint && ka[i] == 2) ? out.x : l0[cu[i] + 1];
                if (kb[i] != 0) o[c1[i] + 2] = (kint && kb[i] == 2) ? out.y : l0[cu[i] + 2];
            }
#pragma unroll
            for (int j = 0; j < PR; ++j) {
                if (rk[j] == 0) continue;
                const int c = ru[j];
                const S* l0 = pls[1];
                S v = l0[c];
                if (kint && rk[j] == 2) {
                    auto ld = [&](int ox, int oy, int oz) -> S {
                        return pls[oz + 1][c + oy * W + ox];
                    };
                    v = jacobi_value<S, 3, Q1>(h2, omega, rb[j], l0[c], ld);
                }
                o[r1[j]] = v;
            }
        }
        __syncthreads();
        if (k - 1 >= z0) {
            const S* pls[3] = {L1[slot(k - 2)], L1[slot(k - 1)], L1[slot(k)]};
            S* dp = dst + (k - 1) * g.sz;
#pragma unroll
            for (int i = 0; i < P; ++i) {
                if (ka[i] != 2) continue;
                const v2 out = q1_jacobi_pair<S, W1>(pls, c1[i], bp2[i], h2v, omv);
                S* p = dp + toff[i];
                if (kb[i] == 2 && (((uintptr_t)p & (2 * sizeof(S) - 1)) == 0)) {
                    __builtin_nontemporal_store(out, reinterpret_cast<v2*>(p));
                } else {
                    st_stream(p, out.x);
                    if (kb[i] == 2) st_stream(p + 1, out.y);
                }
            }
        }
    };
    for (int64_t k = z0 - 1; k <= z1; k += 3) {
        step(k, B0, B2, B1, R0, R1);
        if (k + 1 > z1) break;
        step(k + 1, B1, B0, B2, R1, R2);
        if (k + 2 > z1) break;
        step(k + 2, B2, B1, B0, R2, R0);
    }
}

// Workgroups that fit the device at once for kernel kern (queried once per
// kernel by the caller) and the z-chunking that fills them.
template <typename K>
int64_t resident_of(K kern, int nt)
{
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, nt, 0) != hipSuccess ||
        hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        per_cu = 2;
        cus = 256;
    }
    return (int64_t)(per_cu > 0 ? per_cu : 1) * cus;
}

StreamWork chunk_tiles(const Geo& g, int tx, int ty, int64_t resident)
{
    StreamWork wk;
    wk.tiles_x = (int)((g.nx + tx - 1) / tx);
    wk.tiles_y = (int)((g.ny + ty - 1) / ty);
    const int64_t tiles = (int64_t)wk.tiles_x * wk.tiles_y;
    int64_t chunks = resident / tiles;
    if (chunks < 1) chunks = 1;
    if (chunks > g.nz / 4) chunks = g.nz / 4 > 0 ? g.nz / 4 : 1;
    wk.chunks = (int)chunks;
    wk.nblocks = tiles * chunks;
    return wk;
}

template <typename S, int ST, int MODE, int TX, int TY, int NT>
StreamWork plan(const Geo& g, int max_blocks)
{
    auto kern = k_stream3<S, ST, MODE, TX, TY, NT>;
    StreamWork wk;
    wk.tiles_x = (int)((g.nx + TX - 1) / TX);
    wk.tiles_y = (int)((g.ny + TY - 1) / TY);
    const int64_t tiles = (int64_t)wk.tiles_x * wk.tiles_y;
    static const int64_t resident = resident_of(kern, NT);  // once per kernel
    int64_t chunks = resident / tiles;
    if (chunks < 1) chunks = 1;
    if (chunks > g.nz / 4) chunks = g.nz / 4 > 0 ? g.nz / 4 : 1;
    while (chunks > 1 && tiles * chunks > max_blocks) --chunks;
    wk.chunks = (int)chunks;
    wk.nblocks = tiles * chunks;
    return wk;
}

template <typename S, int ST>
cs_status jacobi3_t(const Geo& g, const void* src, void* dst, const void* b, double h2,
                    double omega, hipStream_t s)
{
    constexpr int TX = 64, TY = 8, NT = 256;
    if (ST == Q1) {
        auto kern = k_jacobi3_q1_pairs<S, TX, TY, NT>;
        static const int64_t resident = resident_of(kern, NT);
        const StreamWork wk = chunk_tiles(g, TX, TY, resident);
        hipLaunchKernelGGL(kern, dim3((unsigned)wk.nblocks), dim3(NT), 0, s, (const S*)src, (S*)dst,
                           (const S*)b, g, h2, omega, wk);
        return check_launch("streaming jacobi (27-point pairs)");
    }
    const StreamWork wk = plan<S, ST, MODE_JACOBI, TX, TY, NT>(g, 1 << 30);
    hipLaunchKernelGGL((k_stream3<S, ST, MODE_JACOBI, TX, TY, NT>), dim3((unsigned)wk.nblocks),
                       dim3(NT), 0, s, (const S*)src, (S*)dst, (const S*)b, g, h2, omega, wk,
                       (Partial*)nullptr, g, (float*)nullptr, (float*)nullptr);
    return check_launch("streaming jacobi");
}

// Two sweeps per launch (the caller pairs the sweeps).  Tile 64 x 16; FP64
// runs best with 512 threads, FP32 with 256 (measured at 256^3).
constexpr int kJ2TX = 64, kJ2TY = 16, kJ2NT64 = 512, kJ2NT32 = 256, kJ2Fill = 1;
constexpr int kJ2QTX = 64, kJ2QTY = 16, kJ2QNT64 = 512, kJ2QNT32 = 256;
template <typename S, int ST>
cs_status jacobi3_two_t(const Geo& g, const void* src, void* dst, const void* b, double h2,
                        double omega, hipStream_t s)
{
    constexpr bool f64 = sizeof(S) == 8;
    if (ST == Q1) {
        constexpr int TX = kJ2QTX, TY = kJ2QTY, NT = f64 ? kJ2QNT64 : kJ2QNT32;
        auto kern = k_jacobi3_q1_two<S, TX, TY, NT>;
        static const int64_t resident = resident_of(kern, NT);
        const StreamWork wk = chunk_tiles(g, TX, TY, resident);
        hipLaunchKernelGGL(kern, dim3((unsigned)wk.nblocks), dim3(NT), 0, s, (const S*)src,
                           (S*)dst, (const S*)b, g, h2, omega, wk);
        return check_launch("streaming jacobi (two sweeps, 27-point)");
    }
    constexpr int TX = kJ2TX, TY = kJ2TY, NT = f64 ? kJ2NT64 : kJ2NT32;
    auto kern = k_jacobi3_fd_two<S, TX, TY, NT>;
    static const int64_t resident = resident_of(kern, NT);
    const StreamWork wk = chunk_tiles(g, TX, TY, resident * kJ2Fill);
    hipLaunchKernelGGL(kern, dim3((unsigned)wk.nblocks), dim3(NT), 0, s, (const S*)src, (S*)dst,
                       (const S*)b, g, h2, omega, wk);
    return check_launch("streaming jacobi (two sweeps, 7-point)");
}

template <typename S, int ST>
cs_status residual3_t(const Geo& g, const void* u, const void* b, void* r, double h2,
                      Partial* partials, double* norms, hipStream_t s)
{
    constexpr int TX = 64, TY = 8, NT = 256;
    const StreamWork wk = plan<S, ST, MODE_RESIDUAL, TX, TY, NT>(g, kMaxResidualBlocks);
    if (wk.nblocks > kMaxResidualBlocks) {
        set_error("residual: grid needs more than %d blocks", kMaxResidualBlocks);
        return CS_EUNSUPPORTED;
    }
    hipLaunchKernelGGL((k_stream3<S, ST, MODE_RESIDUAL, TX, TY, NT>), dim3((unsigned)wk.nblocks),
                       dim3(NT), 0, s, (const S*)u, (S*)r, (const S*)b, g, h2, 0.0, wk, partials,
                       g, (float*)nullptr, (float*)nullptr);
    cs_status st = check_launch("streaming residual");
    if (st != CS_OK) return st;
    return launch_residual_finish(partials, (int)wk.nblocks, norms, s);
}

template <int ST>
cs_status ir_residual3_t(const Geo& g, const void* x, const void* b, double h2, double inv_scale,
                         const Geo& g2, void* r32, void* e32, Partial* partials, double* norms,
                         hipStream_t s)
{
    constexpr int TX = 64, TY = 8, NT = 256;
    const StreamWork wk = plan<double, ST, MODE_IR, TX, TY, NT>(g, kMaxResidualBlocks);
    if (wk.nblocks > kMaxResidualBlocks) {
        set_error("ir residual: grid needs more than %d blocks", kMaxResidualBlocks);
        return CS_EUNSUPPORTED;
    }
    hipLaunchKernelGGL((k_stream3<double, ST, MODE_IR, TX, TY, NT>), dim3((unsigned)wk.nblocks),
                       dim3(NT), 0, s, (const double*)x, (double*)nullptr, (const double*)b, g, h2,
                       inv_scale, wk, partials, g2, (float*)r32, (float*)e32);
    cs_status st = check_launch("ir residual");
    if (st != CS_OK) return st;
    return launch_residual_finish(partials, (int)wk.nblocks, norms, s);
}

}  // namespace

cs_status launch_ir_residual3(int stencil, const Geo& g, const void* x, const void* b, double h2,
                              double inv_scale, const Geo& g2, void* r32, void* e32,
                              Partial* partials, double* norms, hipStream_t s)
{
    return stencil == FD
               ? ir_residual3_t<FD>(g, x, b, h2, inv_scale, g2, r32, e32, partials, norms, s)
               : ir_residual3_t<Q1>(g, x, b, h2, inv_scale, g2, r32, e32, partials, norms, s);
}

bool stream_supported(const Geo& g)
{
    return (g.ny + 2) * g.sy < ((int64_t)1 << 31);
}

// The streaming residual keeps one partial per workgroup, at most
// kMaxResidualBlocks of them, and needs one 64 x 8 tile per workgroup at
// least; larger planes take the generic residual, which clamps its grid.
bool residual3_stream_fits(const Geo& g)
{
    const int64_t tiles = ((g.nx + 63) / 64) * ((g.ny + 7) / 8);
    return stream_supported(g) && tiles <= kMaxResidualBlocks;
}

cs_status launch_jacobi3_stream(int dtype, int stencil, const Geo& g, const void* src, void* dst,
                                const void* b, double h2, double omega, hipStream_t s)
{
    if (dtype == 0)
        return stencil == FD ? jacobi3_t<double, FD>(g, src, dst, b, h2, omega, s)
                             : jacobi3_t<double, Q1>(g, src, dst, b, h2, omega, s);
    return stencil == FD ? jacobi3_t<float, FD>(g, src, dst, b, h2, omega, s)
                         : jacobi3_t<float, Q1>(g, src, dst, b, h2, omega, s);
}

bool jacobi3_two_supported(int stencil, const Geo& g)
{
    (void)stencil;
    return stream_supported(g);
}

cs_status launch_jacobi3_two(int dtype, int stencil, const Geo& g, const void* src, void* dst,
                             const void* b, double h2, double omega, hipStream_t s)
{
    if (dtype == 0)
        return stencil == FD ? jacobi3_two_t<double, FD>(g, src, dst, b, h2, omega, s)
                             : jacobi3_two_t<double, Q1>(g, src, dst, b, h2, omega, s);
    return stencil == FD ? jacobi3_two_t<float, FD>(g, src, dst, b, h2, omega, s)
                         : jacobi3_two_t<float, Q1>(g, src, dst, b, h2, omega, s);
}

cs_status launch_residual3_stream(int dtype, int stencil, const Geo& g, const void* u,
                                  const void* b, void* r, double h2, Partial* partials,
                                  double* norms, hipStream_t s)
{
    if (dtype == 0)
        return stencil == FD ? residual3_t<double, FD>(g, u, b, r, h2, partials, norms, s)
                             : residual3_t<double, Q1>(g, u, b, r, h2, partials, norms, s);
    return stencil == FD ? residual3_t<float, FD>(g, u, b, r, h2, partials, norms, s)
                         : residual3_t<float, Q1>(g, u, b, r, h2, partials, norms, s);
}

}  // namespace cs
