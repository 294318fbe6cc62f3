"""Pins of the oracle's discretisation (no GPU).

Each test checks the oracle against a fact fixed by the paper or by the
mathematics of Whitney elements, not against itself."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as W
from oracle import fem


def _system(dims, rule="all", h=None, removed=None, mu=None, gamma=1.0):
    mesh = W.hex_box_mesh(dims, h=h, removed=removed)
    T = mesh["tets"].shape[0]
    mu = np.ones(T) if mu is None else mu
    return fem.System(mesh, mu, np.ones(T), gamma, W.dirichlet_flags(mesh["bface_tag"], rule))


@pytest.mark.parametrize("N,edges,nodes", [(8, 121_696, 18_785), (16, 242_592, 37_281)])
def test_paper_beam_counts(N, edges, nodes):
    """Section 4 (Numerical results), Table 1: the beam N/2 x 1 x 1 at h = 1/16 has 122K / 243K
    dofs (all edges) and NK size 19K / 37K (all nodes) for N = 8 / 16; the
    closed-form counts of the Kuhn-split hex grid are 121,696 / 242,592 edges
    and 18,785 / 37,281 nodes.  The text gives 121,696 exactly."""
    mesh = W.hex_box_mesh((8 * N, 16, 16), h=1.0 / 16)
    e, _ = fem.edge_table(mesh["tets"])
    assert e.shape[0] == edges
    assert mesh["xyz"].shape[0] == nodes
    X, Y, Z = 8 * N, 16, 16
    closed = (X * (Y + 1) * (Z + 1) + (X + 1) * Y * (Z + 1) + (X + 1) * (Y + 1) * Z
              + X * Y * (Z + 1) + X * (Y + 1) * Z + (X + 1) * Y * Z + X * Y * Z)
    assert closed == edges


def test_curl_curl_annihilates_gradients():
    """G is exactly the null space part of the discrete curl-curl matrix
    (Section 1): K G = 0 up to round-off, also on a mesh with a hole, mixed
    boundary conditions and heterogeneous mu."""
    for dims, rule, removed in [((4, 4, 4), "all", None), ((6, 6, 3), "outer", "hole"), ((6, 3, 3), "mixed", None)]:
        rem = None
        if removed == "hole":
            rem = np.zeros(dims, bool)
            rem[2:4, 2:4, :] = True
        mesh = W.hex_box_mesh(dims, removed=rem)
        T = mesh["tets"].shape[0]
        mu = np.exp(np.random.default_rng(0).normal(0, 2, T))
        s = fem.System(mesh, mu, np.ones(T), 1e-3, W.dirichlet_flags(mesh["bface_tag"], rule))
        KG = s.K @ s.G
        assert abs(KG).max() <= 1e-12 * abs(s.K).max()
        # and G has full column rank when a Dirichlet face exists: G^T G SPD
        GtG = (s.G.T @ s.G).toarray()
        assert np.linalg.eigvalsh(GtG).min() > 1e-10


def test_element_constant_and_linear_fields():
    """Whitney interpolation reproduces a + b x x exactly: for a constant
    field c, (Pi c)^T M_e (Pi c) = |T| |c|^2 and K_e Pi c = 0; for
    u = a x x, curl u = 2a and (Pi u)^T K_e (Pi u) = |T| |2a|^2."""
    rng = np.random.default_rng(3)
    for _ in range(5):
        P = rng.normal(size=(4, 3))
        gids = rng.permutation(10)[:4]
        Ke, Me = fem.element_matrices(P, gids)
        _, vol = fem.barycentric_gradients(P)
        ends = [(a, b) if gids[a] < gids[b] else (b, a) for a, b in fem.LOCAL_EDGES]
        c = rng.normal(size=3)
        pic = np.array([c @ (P[b] - P[a]) for a, b in ends])
        assert np.isclose(pic @ Me @ pic, vol * c @ c, rtol=1e-12)
        assert np.allclose(Ke @ pic, 0, atol=1e-12 * abs(Ke).max())
        a3 = rng.normal(size=3)
        # line integral of a x x along a->b (linear field: midpoint rule exact)
        piu = np.array([np.cross(a3, 0.5 * (P[a] + P[b])) @ (P[b] - P[a]) for a, b in ends])
        assert np.isclose(piu @ Ke @ piu, vol * 4 * a3 @ a3, rtol=1e-11)
        assert np.allclose(Ke, Ke.T) and np.allclose(Me, Me.T)
        assert np.linalg.eigvalsh(Me).min() > 0


def test_vectorised_elements_match_scalar_formula():
    mesh = W.hex_box_mesh((2, 2, 2))
    Ke, Me = fem.element_matrices_all(mesh["xyz"], mesh["tets"].astype(np.int64))
    for t in range(0, mesh["tets"].shape[0], 7):
        k, m = fem.element_matrices(mesh["xyz"][mesh["tets"][t]], mesh["tets"][t])
        assert np.allclose(Ke[t], k, rtol=1e-14, atol=1e-14)
        assert np.allclose(Me[t], m, rtol=1e-14, atol=1e-14)


def test_manufactured_solution_first_order():
    """E* = (sin py sin pz, sin pz sin px, sin px sin py) satisfies n x E* = 0
    on the unit cube and curl curl E* = 2 pi^2 E*, so f = (2 pi^2 + gamma) E*.
    Lowest-order edge elements converge at first order in L2 and in the curl
    norm (textbook rate)."""
    pi = np.pi

    def Es(x):
        return np.stack([np.sin(pi * x[:, 1]) * np.sin(pi * x[:, 2]),
                         np.sin(pi * x[:, 2]) * np.sin(pi * x[:, 0]),
                         np.sin(pi * x[:, 0]) * np.sin(pi * x[:, 1])], 1)

    def cE(x):
        X, Y, Z = x[:, 0], x[:, 1], x[:, 2]
        s, c = np.sin, np.cos
        return pi * np.stack([s(pi * X) * c(pi * Y) - s(pi * X) * c(pi * Z),
                              s(pi * Y) * c(pi * Z) - c(pi * X) * s(pi * Y),
                              c(pi * X) * s(pi * Z) - c(pi * Y) * s(pi * Z)], 1)
    errs = []
    for m in (4, 8):
        s = _system((m, m, m), gamma=1.0)
        b = fem.load_vector(s, lambda x: (2 * pi ** 2 + 1.0) * Es(x))
        u = spla.spsolve(s.A.tocsc(), b)
        errs.append(fem.l2_errors(s, u, Es, cE))
    r0 = np.log2(errs[0][0] / errs[1][0])
    r1 = np.log2(errs[0][1] / errs[1][1])
    assert 0.85 < r0 < 1.3 and 0.85 < r1 < 1.3, (errs, r0, r1)


def test_system_spd_and_dirichlet_elimination():
    s = _system((4, 4, 4), gamma=1e-3)
    A = s.A.toarray()
    assert np.allclose(A, A.T, atol=1e-15)
    assert np.linalg.eigvalsh(A).min() > 0
    # 4^3 cube: all edges 604... free = interior edges; counts from closed form
    X = 4
    all_e = 3 * X * (X + 1) ** 2 + 3 * X * X * (X + 1) + X ** 3
    assert s.edges.shape[0] == all_e
    assert s.p == (X - 1) ** 3
