// Gauss-Seidel in the nested-dissection ordering (Sec. 3).  The paper cuts the
// domain into 2^d blocks and a one-cell separator, recursively, and runs the
// blocks, which do not couple, before their separator; the recursion depth and
// the order inside a separator are left to the machine.  Reading taken here: a
// box whose every edge is at most `leaf` cells is a leaf, swept in z-y-x order;
// otherwise every axis longer than `leaf` is cut at the cell lo + extent / 2,
// the sub-boxes are processed recursively, then the separator (the cells of the
// box on a cut) in z-y-x order.
//
// Two boxes of the tree that are not nested lie on different sides of the cut
// of their lowest common ancestor, at least two cells apart, so they never
// read each other's cells: every node of one height can run at once.  One
// launch per height (leaves first), one thread (2D) or one workgroup (3D, by
// hyperplanes, below) per node, updating the node's cells in its order with
// the colour-pass update -- Gauss-Seidel in the dissection ordering, the
// oracle's iterate bit for bit.  The tree is built on the host, once per grid
// and leaf size.
#include "cs_device.h"
#include "cs_internal.h"

#include <algorithm>
#include <vector>

namespace cs {

namespace {

template <typename T, int DIM, int ST>
__global__ void __launch_bounds__(64)
k_nd_stage(T* u, const T* __restrict__ b, Geo g, T h2, const NdNode* __restrict__ nodes, int count)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    const NdNode nd = nodes[t];
    const int64_t sy = g.sy, sz = g.sz;
    auto upd = [&](int64_t i, int64_t j, int64_t k) {
        const int64_t q = (DIM == 3 ? k * sz : 0) + j * sy + i;
        auto ld = [&](int ox, int oy, int oz) { return u[q + oz * sz + oy * sy + ox]; };
        u[q] = gs_value<T, DIM, ST>(h2, b[q], ld);
    };
    if (nd.cut == 0) {
        for (int64_t k = nd.lo[2]; k <= nd.hi[2]; ++k)
            for (int64_t j = nd.lo[1]; j <= nd.hi[1]; ++j)
                for (int64_t i = nd.lo[0]; i <= nd.hi[0]; ++i) upd(i, j, k);
        return;
    }
    // the cells on a cut, z-y-x order
    for (int64_t k = nd.lo[2]; k <= nd.hi[2]; ++k) {
        if ((nd.cut & 4) && k == nd.m[2]) {
            for (int64_t j = nd.lo[1]; j <= nd.hi[1]; ++j)
                for (int64_t i = nd.lo[0]; i <= nd.hi[0]; ++i) upd(i, j, k);
            continue;
        }
        for (int64_t j = nd.lo[1]; j <= nd.hi[1]; ++j) {
            if ((nd.cut & 2) && j == nd.m[1]) {
                for (int64_t i = nd.lo[0]; i <= nd.hi[0]; ++i) upd(i, j, k);
                continue;
            }
            if (nd.cut & 1) upd(nd.m[0], j, k);
        }
    }
}

// The same stage with one workgroup per node: the node's cells are updated by
// hyperplanes s = wx i + wy j + wz k in increasing s, every cell of one
// hyperplane at once, a workgroup barrier between hyperplanes.  The weights
// (1, 1, 1) for the 2d+1-point and (1, 2, 4) for the 3^d-point stencils put
// every neighbour that precedes a cell in z-y-x order on a smaller s and every
// later one on a larger s (as in the lexicographic wavefront sweep), and the
// cells outside the node do not change while it runs, so this is the node's
// z-y-x order, bit for bit, without a dependent chain per thread.
constexpr int kNdThreads = 256;

template <typename T, int DIM, int ST>
__global__ void __launch_bounds__(kNdThreads)
k_nd_stage_wg(T* u, const T* __restrict__ b, Geo g, T h2, const NdNode* __restrict__ nodes)
{
    constexpr int64_t WX = 1, WY = ST == FD ? 1 : 2, WZ = DIM == 3 ? (ST == FD ? 1 : 4) : 0;
    const NdNode nd = nodes[blockIdx.x];
    const int64_t sy = g.sy, sz = g.sz;
    auto upd = [&](int64_t i, int64_t j, int64_t k) {
        const int64_t q = (DIM == 3 ? k * sz : 0) + j * sy + i;
        auto ld = [&](int ox, int oy, int oz) { return u[q + oz * sz + oy * sy + ox]; };
        u[q] = gs_value<T, DIM, ST>(h2, b[q], ld);
    };
    const int64_t lo0 = nd.lo[0], lo1 = nd.lo[1], lo2 = nd.lo[2];
    const int64_t hi0 = nd.hi[0], hi1 = nd.hi[1], hi2 = nd.hi[2];
    const int64_t ny = hi1 - lo1 + 1, nz = hi2 - lo2 + 1;
    const int64_t smin = WX * lo0 + WY * lo1 + WZ * lo2, smax = WX * hi0 + WY * hi1 + WZ * hi2;
    const bool cx = nd.cut & 1, cy = (nd.cut >> 1) & 1, cz = (nd.cut >> 2) & 1;
    for (int64_t sv = smin; sv <= smax; ++sv) {
        if (nd.cut == 0) {
            // leaf: every (j, k) row holds at most one cell of the hyperplane
            for (int64_t r = threadIdx.x; r < ny * nz; r += blockDim.x) {
                const int64_t j = lo1 + r % ny, k = lo2 + r / ny;
                const int64_t i = sv - WY * j - WZ * k;
                if (i >= lo0 && i <= hi0) upd(i, j, k);
            }
        } else {
            // the separator, each cell once: the plane k = m2 (one cell per row
            // j), the plane j = m1 without k = m2 (one per k), the plane i = m0
            // without j = m1 and k = m2 (at most one per k)
            const int64_t np = cz ? ny : 0, nq = cy ? nz : 0, nr = cx ? nz : 0;
            for (int64_t t = threadIdx.x; t < np + nq + nr; t += blockDim.x) {
                int64_t i, j, k;
                if (t < np) {
                    j = lo1 + t;
                    k = nd.m[2];
                } else if (t < np + nq) {
                    k = lo2 + (t - np);
                    j = nd.m[1];
                    if (cz && k == nd.m[2]) continue;
                } else {
                    k = lo2 + (t - np - nq);
                    i = nd.m[0];
                    const int64_t rem = sv - WX * i - WZ * k;
                    if (rem % WY != 0) continue;
                    j = rem / WY;
                    if (j < lo1 || j > hi1 || (cy && j == nd.m[1]) || (cz && k == nd.m[2])) continue;
                    upd(i, j, k);
                    continue;
                }
                i = sv - WY * j - WZ * k;
                if (i >= lo0 && i <= hi0) upd(i, j, k);
            }
        }
        __syncthreads();
    }
}

// Append the subtree of box [lo, hi] to out (with each node's height) and
// return its height.
int build(const int32_t* lo, const int32_t* hi, int dim, int64_t leaf, std::vector<NdNode>& out,
          std::vector<int>& height)
{
    NdNode nd;
    nd.cut = 0;
    for (int a = 0; a < 3; ++a) {
        nd.lo[a] = lo[a];
        nd.hi[a] = hi[a];
        nd.m[a] = 0;
        const int64_t ext = (int64_t)hi[a] - lo[a] + 1;
        if (a < dim && ext > leaf) {
            nd.cut |= 1 << a;
            nd.m[a] = (int32_t)(lo[a] + ext / 2);
        }
    }
    int h = -1;
    if (nd.cut) {
        for (int hz = 0; hz <= ((nd.cut >> 2) & 1); ++hz)
            for (int hy = 0; hy <= ((nd.cut >> 1) & 1); ++hy)
                for (int hx = 0; hx <= (nd.cut & 1); ++hx) {
                    const int half[3] = {hx, hy, hz};
                    int32_t clo[3], chi[3];
                    bool empty = false;
                    for (int a = 0; a < 3; ++a) {
                        clo[a] = lo[a];
                        chi[a] = hi[a];
                        if ((nd.cut >> a) & 1) {
                            if (half[a] == 0) chi[a] = nd.m[a] - 1;
                            else clo[a] = nd.m[a] + 1;
                        }
                        empty = empty || clo[a] > chi[a];
                    }
                    if (!empty) h = std::max(h, build(clo, chi, dim, leaf, out, height));
                }
    }
    out.push_back(nd);
    height.push_back(h + 1);
    return h + 1;
}

template <typename T, int DIM, int ST>
cs_status nd_t(const Geo& g, void* u, const void* b, double h2, int nsweeps, const NdNode* nodes,
               const int* stage_off, int nstages, hipStream_t s)
{
    for (int sw = 0; sw < nsweeps; ++sw)
        for (int st = 0; st < nstages; ++st) {
            const int off = stage_off[st], cnt = stage_off[st + 1] - off;
            // 2D nodes are small (a leaf row, a separator line): a chain per
            // thread beats a barrier per hyperplane; 3D separators are planes
            if (DIM == 2)
                hipLaunchKernelGGL((k_nd_stage<T, DIM, ST>), dim3((unsigned)((cnt + 63) / 64)), dim3(64), 0, s,
                                   (T*)u, (const T*)b, g, (T)h2, nodes + off, cnt);
            else
                hipLaunchKernelGGL((k_nd_stage_wg<T, DIM, ST>), dim3((unsigned)cnt), dim3(kNdThreads), 0, s,
                                   (T*)u, (const T*)b, g, (T)h2, nodes + off);
            const cs_status e = check_launch("nested-dissection stage");
            if (e != CS_OK) return e;
        }
    return CS_OK;
}

}  // namespace

cs_status nd_tree(const Geo& g, int dim, int64_t leaf, std::vector<NdNode>* nodes,
                  std::vector<int>* stage_off)
{
    std::vector<NdNode> out;
    std::vector<int> height;
    const int32_t lo[3] = {1, 1, 1};
    const int32_t hi[3] = {(int32_t)g.nx, (int32_t)g.ny, (int32_t)(dim == 3 ? g.nz : 1)};
    const int top = build(lo, hi, dim, leaf, out, height);
    // nodes grouped by height, leaves first
    std::vector<int> idx(out.size());
    for (size_t i = 0; i < idx.size(); ++i) idx[i] = (int)i;
    std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return height[x] < height[y]; });
    nodes->clear();
    stage_off->assign((size_t)top + 2, 0);
    for (int i : idx) {
        nodes->push_back(out[i]);
        ++(*stage_off)[(size_t)height[i] + 1];
    }
    for (size_t h = 1; h < stage_off->size(); ++h) (*stage_off)[h] += (*stage_off)[h - 1];
    return CS_OK;
}

cs_status launch_nd_sweeps(int dtype, int dim, int stencil, const Geo& g, void* u, const void* b,
                           double h2, int nsweeps, const NdNode* nodes, const int* stage_off,
                           int nstages, hipStream_t s)
{
    if (dtype == 0) {
        if (dim == 2)
            return stencil == FD ? nd_t<double, 2, FD>(g, u, b, h2, nsweeps, nodes, stage_off, nstages, s)
                                 : nd_t<double, 2, Q1>(g, u, b, h2, nsweeps, nodes, stage_off, nstages, s);
        return stencil == FD ? nd_t<double, 3, FD>(g, u, b, h2, nsweeps, nodes, stage_off, nstages, s)
                             : nd_t<double, 3, Q1>(g, u, b, h2, nsweeps, nodes, stage_off, nstages, s);
    }
    if (dim == 2)
        return stencil == FD ? nd_t<float, 2, FD>(g, u, b, h2, nsweeps, nodes, stage_off, nstages, s)
                             : nd_t<float, 2, Q1>(g, u, b, h2, nsweeps, nodes, stage_off, nstages, s);
    return stencil == FD ? nd_t<float, 3, FD>(g, u, b, h2, nsweeps, nodes, stage_off, nstages, s)
                         : nd_t<float, 3, Q1>(g, u, b, h2, nsweeps, nodes, stage_off, nstages, s);
}

}  // namespace cs
