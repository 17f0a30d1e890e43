// Device-side stencil helpers shared by the colsten kernels.
//
// The dimensionless stencils of the 2d+1-point finite-difference family and
// the 3^d-point d-linear finite-element family (Fig. 1 and Sec. 2 of
// Hazelwood & Weinzierl, arXiv:1810.04033; the 27-point entries are the
// assembled trilinear element stiffness: faces 0, edges -1/6, corners -1/12).
//
// The library is compiled with -ffp-contract=off, so the only fused
// operations are the explicit fused multiply-adds below.  Neighbour sums visit
// the offsets in lexicographic (oz, oy, ox) order, skip zero weights and add
// each term with one fused multiply-add (acc <- fma(S_o, u_{q+o}, acc)), so a
// kernel using these helpers rounds exactly like a plain sequential
// evaluation of
//     u_q <- (h^2 b_q - sum_{o != 0} S_o u_{q+o}) / S_0
// written the same way, with the quotient by S_0 formed as in over_centre.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cs {

enum { FD = 0, Q1 = 1 };

// S_o for offset (ox, oy, oz).  Weights are formed in T's own arithmetic
// (T(-1) / T(6) is the correctly rounded quotient in T).
template <typename T, int DIM, int ST>
__host__ __device__ constexpr T weight(int ox, int oy, int oz)
{
    const int nnz = (ox != 0) + (oy != 0) + (oz != 0);
    if (DIM == 2 && oz != 0) return T(0);
    if (ST == FD) return nnz == 0 ? T(2 * DIM) : (nnz == 1 ? T(-1) : T(0));
    if (DIM == 2) return nnz == 0 ? T(8) / T(3) : T(-1) / T(3);
    return nnz == 0 ? T(8) / T(3)
         : nnz == 1 ? T(0)
         : nnz == 2 ? T(-1) / T(6)
                    : T(-1) / T(12);
}

template <int ST, int DIM>
__host__ __device__ constexpr int num_colours()
{
    return ST == FD ? 2 : (1 << DIM);
}

// Store of a value that no thread of the same launch reads again (the new
// iterate of a sweep): a nontemporal store, which keeps the caches for the
// halo rows that neighbouring tiles re-read.
template <typename T>
__device__ __forceinline__ void st_stream(T* p, T v)
{
    __builtin_nontemporal_store(v, p);
}

__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// sum_{o} S_o * ld(ox, oy, oz) over the nonzero weights, lexicographic
// (oz, oy, ox) order; the centre is included iff CENTRE.
template <typename T, int DIM, int ST, bool CENTRE, typename Load>
__device__ __forceinline__ T ordered_sum(const Load& ld)
{
    T acc = T(0);
#pragma unroll
    for (int oz = (DIM == 3 ? -1 : 0); oz <= (DIM == 3 ? 1 : 0); ++oz) {
#pragma unroll
        for (int oy = -1; oy <= 1; ++oy) {
#pragma unroll
            for (int ox = -1; ox <= 1; ++ox) {
                if (!CENTRE && ox == 0 && oy == 0 && oz == 0) continue;
                const T w = weight<T, DIM, ST>(ox, oy, oz);
                if (w == T(0)) continue;
                acc = fma_t(w, (T)ld(ox, oy, oz), acc);
            }
        }
    }
    return acc;
}

// x / S_0 as the exact quotient rounded once.
//  - d-linear stencils: S_0 = 8/3 has the binary inverse 3/8, so the quotient
//    is the product x * 0.375.
//  - 2D FD: S_0 = 4, a power of two: x * 0.25 is the quotient.
//  - 3D FD: S_0 = 6.  q = RN(x z) with z = RN(1/6) is within two ulps of
//    x/6, so the residual r = x - 6q is exact in one fused multiply-add, and
//    q' = RN(q + r z) = RN(x/6 + e) with |e| <= |r| |z - 1/6|, about
//    2^-p ulp(x/6) (p = 53 or 24).  For a divisor 3 * 2^k the exact quotient
//    of a p-bit x lies at least ulp(x/6) / 6 away from every rounding
//    midpoint (|8m - 3(2k+1)| >= 1 for integers m, k), so q' = RN(x/6) for
//    every x whose quotient is normal, up to the sign of a zero result: three
//    operations instead of a full division (Markstein's correction step for
//    a constant divisor).
template <typename T, int DIM, int ST>
__device__ __forceinline__ T over_centre(T x)
{
    if (ST == Q1) return x * T(0.375);
    if (DIM == 2) return x * T(0.25);
    constexpr T z = T(1) / T(6);
    const T q = x * z;
    const T r = fma_t(-q, T(6), x);
    return fma_t(r, z, q);
}

// Gauss-Seidel value of one point from its neighbours (centre excluded).
template <typename T, int DIM, int ST, typename Load>
__device__ __forceinline__ T gs_value(T h2, T bq, const Load& ld)
{
    const T rhs = h2 * bq;
    const T acc = ordered_sum<T, DIM, ST, false>(ld);
    return over_centre<T, DIM, ST>(rhs - acc);
}

// Weighted Jacobi value: u_q + omega * (h^2 b_q - sum_o S_o u_{q+o}) / S_0,
// the last multiply-add fused.
template <typename T, int DIM, int ST, typename Load>
__device__ __forceinline__ T jacobi_value(T h2, T omega, T bq, T uq, const Load& ld)
{
    const T su = ordered_sum<T, DIM, ST, true>(ld);
    return fma_t(omega, over_centre<T, DIM, ST>(h2 * bq - su), uq);
}

}  // namespace cs
