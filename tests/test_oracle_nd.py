"""Pins of the oracle's nested-dissection sweep (Sec. 3, with the reading
stated in the oracle: leaves of edge <= leaf swept in z-y-x order, cuts at
lo + extent / 2, children before their separator, separator cells in z-y-x
order).  The references are a dense triangular solve in the dissection
ordering, built here from the reading by separate code, the lexicographic
sweep for a single leaf, and the independence of sibling blocks."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1810_04033_amd import inputs as I

import bruteforce as BF


def nd_order(n, leaf, children_reversed=False):
    """Lexicographic interior indices (x fastest) in dissection order."""
    dim = len(n)
    nn = list(n) + [1] * (3 - dim)

    def lin(i, j, k):
        return ((k - 1) * nn[1] + (j - 1)) * nn[0] + (i - 1)

    out = []

    def box(lo, hi):
        cuts = {a: lo[a] + (hi[a] - lo[a] + 1) // 2 for a in range(dim) if hi[a] - lo[a] + 1 > leaf}
        if cuts:
            halves = [(0, 1) if a in cuts else (0,) for a in range(3)]
            kids = []
            for hz in halves[2]:
                for hy in halves[1]:
                    for hx in halves[0]:
                        clo, chi = list(lo), list(hi)
                        for a, hf in ((0, hx), (1, hy), (2, hz)):
                            if a in cuts:
                                if hf == 0:
                                    chi[a] = cuts[a] - 1
                                else:
                                    clo[a] = cuts[a] + 1
                        if all(clo[a] <= chi[a] for a in range(3)):
                            kids.append((clo, chi))
            for clo, chi in (reversed(kids) if children_reversed else kids):
                box(clo, chi)
        for k in range(lo[2], hi[2] + 1):
            for j in range(lo[1], hi[1] + 1):
                for i in range(lo[0], hi[0] + 1):
                    c = (i, j, k)
                    if not cuts or any(c[a] == m for a, m in cuts.items()):
                        out.append(lin(i, j, k))

    box([1, 1, 1], nn)
    return out


CASES = [((20, 13), 4), ((9, 7, 10), 3), ((16, 16), 3), ((12, 5, 7), 2)]


@pytest.mark.parametrize("n,leaf", CASES, ids=lambda p: "x".join(map(str, p)) if isinstance(p, tuple) else str(p))
@pytest.mark.parametrize("stencil", [O.FD, O.Q1], ids=["fd", "q1"])
def test_nd_sweep_is_gauss_seidel_in_the_dissection_order(n, leaf, stencil):
    dim = len(n)
    order = nd_order(n, leaf)
    assert sorted(order) == list(range(int(np.prod(n))))  # every cell once
    h = 1.0 / (max(n) + 1)
    shape = tuple(reversed(n))
    u = I.halo_array(I.uniform_field(41, shape))
    u[(0,) * dim] = 0.0
    b = I.halo_array(I.uniform_field(42, shape))
    want = BF.gs_sweep_order(u.ravel().copy(), b[(slice(1, -1),) * dim].ravel(), dim, stencil, n, h, order)
    want = BF.gs_sweep_order(want, b[(slice(1, -1),) * dim].ravel(), dim, stencil, n, h, order)
    got = u.copy()
    O.nd_sweeps(got, b, 2, dim=dim, stencil=stencil, h=h, leaf=leaf)
    err = np.max(np.abs(got.ravel() - want)) / np.max(np.abs(want))
    assert err <= 1e-12
    # and it is not the lexicographic or the coloured iterate
    lex = u.copy()
    O.lex_sweeps(lex, b, 2, dim=dim, stencil=stencil, h=h)
    assert np.max(np.abs(lex - got)) > 1e-8


def test_sibling_blocks_do_not_couple():
    # running the sub-boxes of every cut in the opposite order is the same sweep
    n, leaf, dim = (14, 11, 9), 3, 3
    h = 1.0 / 15
    shape = tuple(reversed(n))
    u = I.halo_array(I.uniform_field(43, shape))
    bi = I.uniform_field(44, shape).ravel()
    for st in (O.FD, O.Q1):
        a = BF.gs_sweep_order(u.ravel().copy(), bi, dim, st, n, h, nd_order(n, leaf))
        r = BF.gs_sweep_order(u.ravel().copy(), bi, dim, st, n, h, nd_order(n, leaf, children_reversed=True))
        assert np.max(np.abs(a - r)) <= 1e-13 * np.max(np.abs(a))
        assert nd_order(n, leaf) != nd_order(n, leaf, children_reversed=True)


@pytest.mark.parametrize("stencil", [O.FD, O.Q1])
def test_single_leaf_is_lexicographic(stencil):
    n = (7, 6, 5)
    h = 1.0 / 8
    u, b = I.halo_array(I.uniform_field(45, (5, 6, 7))), I.halo_array(I.uniform_field(46, (5, 6, 7)))
    a, c = u.copy(), u.copy()
    O.nd_sweeps(a, b, 3, dim=3, stencil=stencil, h=h, leaf=7)
    O.lex_sweeps(c, b, 3, dim=3, stencil=stencil, h=h)
    assert np.array_equal(a, c)
