"""Dense brute force for tiny grids (tests only; independent of the oracle).

The dimensionless operators are assembled from textbook 1D building blocks by
Kronecker products over the lexicographic interior ordering (x fastest):

* finite differences:  S = sum_m I x .. x T_m x .. x I with T = tridiag(-1, 2, -1)
* d-linear elements:   S = sum_m M x .. x K_m x .. x M with K = tridiag(-1, 2, -1)
  and M = tridiag(1, 4, 1) / 6 (the 1D stiffness and mass of linear elements
  on unit cells), i.e. the tensor-product form of the Q1 stiffness.

Rows cover interior points; columns cover the extended (halo'd) grid so that
Dirichlet values in the halo enter as they do in the stencil form.
"""
import numpy as np
import scipy.linalg as sla


def _ext_1d(n, kind):
    """n x (n+2) matrix acting on a 1D line with halo: interior rows."""
    a = np.zeros((n, n + 2))
    for i in range(n):
        if kind == "K":
            a[i, i], a[i, i + 1], a[i, i + 2] = -1.0, 2.0, -1.0
        elif kind == "M":
            a[i, i], a[i, i + 1], a[i, i + 2] = 1.0 / 6, 4.0 / 6, 1.0 / 6
        elif kind == "I":
            a[i, i + 1] = 1.0
    return a


def _kron(mats):
    out = mats[0]
    for m in mats[1:]:
        out = np.kron(out, m)
    return out


def operator_ext(dim, stencil, n):
    """Dimensionless S on interior rows x extended columns.  n = (nx, ny[, nz])."""
    ns = list(n)[:dim]
    terms = []
    for m in range(dim):  # axis m gets K (or T), the others I (FD) or M (Q1)
        mats = []
        for ax in reversed(range(dim)):  # z, y, x order for x-fastest kron
            if ax == m:
                mats.append(_ext_1d(ns[ax], "K"))
            else:
                mats.append(_ext_1d(ns[ax], "I" if stencil == 0 else "M"))
        terms.append(_kron(mats))
    return sum(terms)


def ext_index(dim, n):
    """Flat extended-grid index of every interior point, lexicographic."""
    nx, ny = n[0], n[1]
    if dim == 2:
        j, i = np.meshgrid(np.arange(1, ny + 1), np.arange(1, nx + 1), indexing="ij")
        return (j * (nx + 2) + i).ravel()
    nz = n[2]
    k, j, i = np.meshgrid(np.arange(1, nz + 1), np.arange(1, ny + 1), np.arange(1, nx + 1), indexing="ij")
    return ((k * (ny + 2) + j) * (nx + 2) + i).ravel()


def split(dim, stencil, n):
    """(A_II, A_IB, interior_cols, boundary_cols) of the dimensionless S."""
    s = operator_ext(dim, stencil, n)
    cols = ext_index(dim, n)
    mask = np.zeros(s.shape[1], dtype=bool)
    mask[cols] = True
    return s[:, cols], s[:, ~mask], cols, np.nonzero(~mask)[0]


def colours(dim, stencil, n, parity):
    """Colour of each interior point, lexicographic order (textbook rules)."""
    nx, ny = n[0], n[1]
    nz = n[2] if dim == 3 else 1
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    if stencil == 0:
        c = (i + j + (k if dim == 3 else 0) + parity) % 2
    else:
        c = (i + parity) % 2 + 2 * ((j + parity) % 2)
        if dim == 3:
            c = c + 4 * ((k + parity) % 2)
    return c.ravel()


def gs_sweep(u_ext_flat, b_int, dim, stencil, n, h, parity):
    """One multicolour Gauss-Seidel sweep by a triangular solve.

    Order the interior unknowns colour-major; with D + L the lower triangle
    (diagonal included) and U the strict upper triangle of the permuted A_II,
    the sweep solves (D + L) u_new = h^2 b - A_IB g - U u_old."""
    a_ii, a_ib, cols, bcols = split(dim, stencil, n)
    col = colours(dim, stencil, n, parity)
    perm = np.argsort(col, kind="stable")
    ap = a_ii[np.ix_(perm, perm)]
    rhs = h * h * b_int - a_ib @ u_ext_flat[bcols]
    u_old = u_ext_flat[cols][perm]
    lower = np.tril(ap)
    upper = ap - lower
    u_new = sla.solve_triangular(lower, rhs[perm] - upper @ u_old, lower=True)
    out = u_ext_flat.copy()
    out[cols[perm]] = u_new
    return out


def gs_sweep_lex(u_ext_flat, b_int, dim, stencil, n, h):
    """One lexicographic Gauss-Seidel sweep: (D + L) u_new = h^2 b - A_IB g - U u_old
    in the natural (x fastest) ordering."""
    a_ii, a_ib, cols, bcols = split(dim, stencil, n)
    rhs = h * h * b_int - a_ib @ u_ext_flat[bcols]
    lower = np.tril(a_ii)
    upper = a_ii - lower
    u_new = sla.solve_triangular(lower, rhs - upper @ u_ext_flat[cols], lower=True)
    out = u_ext_flat.copy()
    out[cols] = u_new
    return out


def gs_sweep_order(u_ext_flat, b_int, dim, stencil, n, h, order):
    """One Gauss-Seidel sweep in an arbitrary ordering of the interior unknowns
    (order: lexicographic interior indices in update order), by the triangular
    solve (D + L) u_new = h^2 b - A_IB g - U u_old of the permuted A_II."""
    a_ii, a_ib, cols, bcols = split(dim, stencil, n)
    perm = np.asarray(order)
    ap = a_ii[np.ix_(perm, perm)]
    rhs = h * h * b_int - a_ib @ u_ext_flat[bcols]
    lower = np.tril(ap)
    upper = ap - lower
    u_new = sla.solve_triangular(lower, rhs[perm] - upper @ u_ext_flat[cols][perm], lower=True)
    out = u_ext_flat.copy()
    out[cols[perm]] = u_new
    return out


def residual(u_ext_flat, b_int, dim, stencil, n, h):
    s = operator_ext(dim, stencil, n)
    return b_int - (s @ u_ext_flat) / (h * h)


def jacobi_sweep(u_ext_flat, b_int, dim, stencil, n, h, omega):
    s = operator_ext(dim, stencil, n)
    a_ii, _, cols, _ = split(dim, stencil, n)
    d = np.diag(a_ii)
    out = u_ext_flat.copy()
    out[cols] = u_ext_flat[cols] + omega * (h * h * b_int - s @ u_ext_flat) / d
    return out
