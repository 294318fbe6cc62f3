"""Pins of the oracle's partitioning, overlap growth, partition of unity and
the constants k0 / k1 (no GPU).

Every expected value below is worked out by hand from the rule the oracle
documents (or from the geometry), not read back from the oracle."""
import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W
from oracle import decomp, fem, geneo


def _system(dims, rule="none", gamma=1.0):
    mesh = W.hex_box_mesh(dims)
    T = mesh["tets"].shape[0]
    return fem.System(mesh, np.ones(T), np.ones(T), gamma, W.dirichlet_flags(mesh["bface_tag"], rule))


# ---------------------------------------------------------------- RCB

def test_rcb_hand_computed_8x2():
    """8x2x1 cells (h = 1, centroids (i+.5, j+.5, .5), id i + 8j) into 3
    parts, jitter (0, 0.2).  Root: widest axis x, 16 cells in (x, id)
    order 0,8,1,9,2,10,...; floor(16/3 + .5) = 5 cells {0,8,1,9,2} -> part 0.
    Right node (11 cells, 2 parts, jitter 0.2): floor(11 * .5 * 1.2 + .5) = 7
    cells {10,3,11,4,12,5,13} -> part 1, {6,14,7,15} -> part 2."""
    mesh = W.hex_box_mesh((8, 2, 1))
    part = decomp.rcb_partition(mesh, 3, [0.0, 0.2])
    expect = np.array([0, 0, 0, 1, 1, 1, 2, 2,
                       0, 0, 1, 1, 1, 1, 2, 2])
    assert np.array_equal(part, expect)


def test_rcb_tie_takes_the_lowest_axis():
    """4x4x1 cells: the x and y extents tie (3 = 3), so the split is along x;
    8 of 16 cells (x < 2) form part 0."""
    mesh = W.hex_box_mesh((4, 4, 1))
    part = decomp.rcb_partition(mesh, 2, [0.0])
    assert np.array_equal(part, np.tile([0, 0, 1, 1], 4))


@pytest.mark.parametrize("j0", [-0.9, 0.9])
def test_rcb_split_is_clipped(j0):
    """3 cells into 3 parts: floor(3 * 1/3 * (1 -+ 0.9) + .5) is 0 or 2, and
    both are clipped to the one cell that leaves every part non-empty."""
    mesh = W.hex_box_mesh((3, 1, 1))
    part = decomp.rcb_partition(mesh, 3, [j0, 0.0])
    assert np.array_equal(part, [0, 1, 2])


# ---------------------------------------------------------------- overlap growth

def test_overlap_layers_grow_by_vertex_adjacency():
    """A single cell (0,0) of a 5x5x1 grid: one layer adds the three cells
    sharing a vertex with it (2x2 block), two layers make a 3x3 block."""
    s = _system((5, 5, 1))
    part = np.ones(25, np.int64)
    part[0] = 0
    ids = lambda block: sorted(i + 5 * j for i in range(block) for j in range(block))
    d1 = decomp.Decomposition(s, part, 1)
    d2 = decomp.Decomposition(s, part, 2)
    assert list(d1.cells[0]) == ids(2)
    assert list(d2.cells[0]) == ids(3)
    assert list(d1.cells[1]) == list(range(25))


# ---------------------------------------------------------------- partition of unity

def _free_edge(s, a, b):
    lo, hi = min(a, b), max(a, b)
    e = np.nonzero((s.edges[:, 0] == lo) & (s.edges[:, 1] == hi))[0]
    assert e.size == 1
    return int(s.edge_to_free[e[0]])


def test_smooth_pou_hand_values():
    """6x1x1 cells (h = 1, no Dirichlet face), two boxes of three cells,
    two overlap layers (eq. (PoU) with the smooth chi of the oracle).
    Part 0 owns x in [0,3]; its layers reach x = 4 (d = 1, chi = 1/2) and
    x = 5 (d = 2, chi = 0).  Part 1 owns [3,6] and reaches x = 2 (chi = 1/2)
    and x = 1 (chi = 0).  An edge's chi is the mean over its ends and
    D_i = chi_i / (chi_0 + chi_1)."""
    s = _system((6, 1, 1))
    dec = decomp.Decomposition(s, decomp.box_partition(s.mesh, (2, 1, 1)), 2)
    nid = lambda i, j, k: i + 7 * (j + 2 * k)
    cases = [
        ((2, 0, 0), (2, 1, 0), 2 / 3, 1 / 3),   # chi (1, 1/2)
        ((3, 0, 0), (4, 0, 0), 3 / 7, 4 / 7),   # chi (3/4, 1)
        ((1, 0, 0), (2, 0, 0), 4 / 5, 1 / 5),   # chi (1, 1/4)
        ((5, 0, 0), (5, 1, 0), 0.0, 1.0),       # chi (0, 1)
        ((0, 0, 0), (1, 0, 0), 1.0, None),      # only in Omega_0
    ]
    for a, b, d0, d1 in cases:
        e = _free_edge(s, nid(*a), nid(*b))
        for i, want in ((0, d0), (1, d1)):
            pos = np.searchsorted(dec.dofs[i], e)
            present = pos < dec.dofs[i].size and dec.dofs[i][pos] == e
            if want is None:
                assert not present
            else:
                assert present and abs(dec.D[i][pos] - want) <= 1e-15, (a, b, i, dec.D[i][pos], want)


def test_paper_snk_count_through_decomposition():
    """Section 4 (Numerical results), Table 1: SNK size 25K for N = 8
    strips of the 64x16x16-hex beam with one overlap layer: the end strips
    are 9 hexes long, the inner ones 10, so the local node counts sum to
    2*10*289 + 6*11*289 = 24,854 (paper convention: every node of every
    subdomain).  Counted on the oracle's own overlapping subdomains."""
    mesh = W.hex_box_mesh((64, 16, 16), h=1.0 / 16)
    T = mesh["tets"].shape[0]
    s = fem.System(mesh, np.ones(T), np.ones(T), 1e-3, W.dirichlet_flags(mesh["bface_tag"], "all"))
    dec = decomp.Decomposition(s, decomp.box_partition(mesh, (8, 1, 1)), 1)
    assert [c.size for c in dec.cells] == [9 * 256] + [10 * 256] * 6 + [9 * 256]
    assert sum(np.unique(mesh["tets"][t]).size for t in dec.tets) == 24_854


# ---------------------------------------------------------------- k0, k1

def test_k0_k1_strips():
    """18x2x2 cells, six strips of three cells, one overlap layer,
    all-Dirichlet.  Strip i covers cells [3i-1, 3i+3].  Strips i and i+1
    overlap; strips i and i+2 are one cell apart, and a Kuhn tet of that
    cell holds a free edge on each of its two faces, so A couples them
    (eq. (k0): R_j A R_i^T != 0); strips three apart are separated by four
    cells.  An inner strip thus meets i-2..i+2: k0 = 5.  No cell lies in
    three strips: k1 = 2."""
    s = _system((18, 2, 2), rule="all")
    dec = decomp.Decomposition(s, decomp.box_partition(s.mesh, (6, 1, 1)), 1)
    assert geneo.k0_k1(dec) == (5, 2)


@pytest.fixture(scope="module")
def cube8():
    w = W.make(1)
    s = fem.System(w.mesh, w.mu, w.eps, w.gamma, w.dirichlet)
    return w, s, decomp.Decomposition(s, decomp.partition_cells(w), w.overlap)


def test_k0_k1_cube8(cube8):
    """2x2x2 boxes of 4^3 cells with one overlap layer: every box meets every
    other (k0 = 8) and the central 2x2x2 cells lie in all eight (k1 = 8)."""
    _, _, dec = cube8
    assert geneo.k0_k1(dec) == (8, 8)


def test_cube8_spectrum_within_main_theorem_bounds(cube8):
    """Main theorem (Section 3.2): spec(M_AS,2^-1 A) lies in
    [1/(1 + k1 tau), k0] = [1/81, 8] for the 8^3 cube (n = 3,032) with no cap
    on the GenEO vectors.  Dense generalised eigenvalues of (A, M) with M^-1
    from the oracle's apply."""
    w, s, dec = cube8
    pre = geneo.TwoLevel(dec, tau=10.0, nev_max=0)
    Minv = pre.matrix()
    Minv = 0.5 * (Minv + Minv.T)
    L = np.linalg.cholesky(Minv)
    ev = sla.eigvalsh(L.T @ s.A.toarray() @ L)
    assert ev[0] >= 1.0 / 81.0 * (1 - 1e-10)
    assert ev[-1] <= 8.0 * (1 + 1e-10)
