// Grid transfers of a geometric multigrid V-cycle whose smoother is the
// coloured Gauss-Seidel sweep (the paper names multigrid as the setting its
// smoothers serve, Sec. 1).  Vertex-centred grids: a fine grid has
// n_f = 2 n_c + 1 interior points per axis and fine index i = 2 I lies on
// coarse index I, so the coarse halo lies on the fine halo.
//
// Restriction by full weighting: at every coarse interior point the 3^d fine
// residuals around 2I, weighted 1/2 on the axis and 1/4 off it per axis, are
// summed in lexicographic (oz, oy, ox) order with one fused multiply-add each;
// the coarse iterate is set to zero at the same point (zero initial guess of
// the coarse correction).  Interpolation: at every fine interior point the
// 1, 2, 4 or 8 coarse values around i/2 (coarse halo included), weighted 1 or
// 1/2 per axis, summed in increasing (cz, cy, cx) order with one fused
// multiply-add each, then added to the fine iterate.  All weights are powers
// of two, so the weight products are exact; one thread per output point, rows
// of 64 points per wavefront.  Each output is a plain function of its inputs,
// so the transfers are deterministic.
#include "cs_device.h"
#include "cs_internal.h"

namespace cs {

namespace {

constexpr int kMX = 64;  // points along x (one wavefront)
constexpr int kMY = 4;   // rows per block

template <typename T, int DIM>
__global__ void __launch_bounds__(kMX* kMY)
k_restrict(const T* __restrict__ r, Geo gf, T* __restrict__ bc, T* __restrict__ uc, Geo gc)
{
    const int64_t I = 1 + (int64_t)blockIdx.x * kMX + threadIdx.x;
    const int64_t J = 1 + (int64_t)blockIdx.y * kMY + threadIdx.y;
    const int64_t K = 1 + (int64_t)blockIdx.z;
    if (I > gc.nx || J > gc.ny) return;
    const int64_t qf = (DIM == 3 ? 2 * K * gf.sz : 0) + 2 * J * gf.sy + 2 * I;
    constexpr int ZR = DIM == 3 ? 1 : 0;
    T acc = T(0);
#pragma unroll
    for (int oz = -ZR; oz <= ZR; ++oz)
#pragma unroll
        for (int oy = -1; oy <= 1; ++oy)
#pragma unroll
            for (int ox = -1; ox <= 1; ++ox) {
                const T wz = DIM == 3 ? (oz == 0 ? T(0.5) : T(0.25)) : T(1);
                const T w = wz * (oy == 0 ? T(0.5) : T(0.25)) * (ox == 0 ? T(0.5) : T(0.25));
                acc = fma_t(w, r[qf + oz * gf.sz + oy * gf.sy + ox], acc);
            }
    const int64_t qc = (DIM == 3 ? K * gc.sz : 0) + J * gc.sy + I;
    bc[qc] = acc;
    uc[qc] = T(0);
}

template <typename T, int DIM>
__global__ void __launch_bounds__(kMX* kMY)
k_prolong_add(const T* __restrict__ uc, Geo gc, T* __restrict__ uf, Geo gf)
{
    const int64_t i = 1 + (int64_t)blockIdx.x * kMX + threadIdx.x;
    const int64_t j = 1 + (int64_t)blockIdx.y * kMY + threadIdx.y;
    const int64_t k = 1 + (int64_t)blockIdx.z;
    if (i > gf.nx || j > gf.ny) return;
    // coarse neighbours along an axis: t/2, and t/2 + 1 when t is odd.  All
    // 2^d candidates (t/2 + 1 <= n_c + 1 stays inside the coarse array) are
    // loaded at once, and only the neighbours enter the ordered sum.
    const bool oz = DIM == 3 && (k & 1), oy = (j & 1) != 0, ox = (i & 1) != 0;
    const T w = (oz ? T(0.5) : T(1)) * (oy ? T(0.5) : T(1)) * (ox ? T(0.5) : T(1));
    const int64_t c0 = (DIM == 3 ? (k / 2) * gc.sz : 0) + (j / 2) * gc.sy + i / 2;
    constexpr int NZ = DIM == 3 ? 2 : 1;
    T v[NZ][2][2];
#pragma unroll
    for (int a = 0; a < NZ; ++a)
#pragma unroll
        for (int bb = 0; bb < 2; ++bb)
#pragma unroll
            for (int c = 0; c < 2; ++c) v[a][bb][c] = uc[c0 + a * gc.sz + bb * gc.sy + c];
    T acc = T(0);
#pragma unroll
    for (int a = 0; a < NZ; ++a)
#pragma unroll
        for (int bb = 0; bb < 2; ++bb)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const bool in = (a == 0 || oz) && (bb == 0 || oy) && (c == 0 || ox);
                acc = in ? fma_t(w, v[a][bb][c], acc) : acc;
            }
    const int64_t q = (DIM == 3 ? k * gf.sz : 0) + j * gf.sy + i;
    uf[q] = uf[q] + acc;
}

// blocks of kMX x kMY points of one plane, one grid layer per plane
bool point_grid(const Geo& g, dim3* grid)
{
    const int64_t gx = (g.nx + kMX - 1) / kMX, gy = (g.ny + kMY - 1) / kMY, gz = g.nz;
    if (gx > 0x7fffffff || gy > 65535 || gz > 65535) return false;
    *grid = dim3((unsigned)gx, (unsigned)gy, (unsigned)gz);
    return true;
}

}  // namespace

cs_status launch_restrict(int dtype, int dim, const Geo& gf, const void* r, const Geo& gc,
                          void* bc, void* uc, hipStream_t s)
{
    dim3 grid;
    if (!point_grid(gc, &grid)) { set_error("restrict: grid too large"); return CS_EUNSUPPORTED; }
    const dim3 block(kMX, kMY);
    if (dtype == 0) {
        if (dim == 3)
            hipLaunchKernelGGL((k_restrict<double, 3>), grid, block, 0, s, (const double*)r, gf,
                               (double*)bc, (double*)uc, gc);
        else
            hipLaunchKernelGGL((k_restrict<double, 2>), grid, block, 0, s, (const double*)r, gf,
                               (double*)bc, (double*)uc, gc);
    } else {
        if (dim == 3)
            hipLaunchKernelGGL((k_restrict<float, 3>), grid, block, 0, s, (const float*)r, gf,
                               (float*)bc, (float*)uc, gc);
        else
            hipLaunchKernelGGL((k_restrict<float, 2>), grid, block, 0, s, (const float*)r, gf,
                               (float*)bc, (float*)uc, gc);
    }
    return check_launch("restriction");
}

cs_status launch_prolong_add(int dtype, int dim, const Geo& gc, const void* uc, const Geo& gf,
                             void* uf, hipStream_t s)
{
    dim3 grid;
    if (!point_grid(gf, &grid)) { set_error("interpolation: grid too large"); return CS_EUNSUPPORTED; }
    const dim3 block(kMX, kMY);
    if (dtype == 0) {
        if (dim == 3)
            hipLaunchKernelGGL((k_prolong_add<double, 3>), grid, block, 0, s, (const double*)uc, gc,
                               (double*)uf, gf);
        else
            hipLaunchKernelGGL((k_prolong_add<double, 2>), grid, block, 0, s, (const double*)uc, gc,
                               (double*)uf, gf);
    } else {
        if (dim == 3)
            hipLaunchKernelGGL((k_prolong_add<float, 3>), grid, block, 0, s, (const float*)uc, gc,
                               (float*)uf, gf);
        else
            hipLaunchKernelGGL((k_prolong_add<float, 2>), grid, block, 0, s, (const float*)uc, gc,
                               (float*)uf, gf);
    }
    return check_launch("interpolation");
}

}  // namespace cs
