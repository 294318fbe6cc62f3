"""Oracle: lowest-order Nedelec (Whitney) discretisation of the positive
Maxwell problem, A = K + gamma*M over free edges, and the gradient matrix G.

Paper passages: the boundary value problem and the discrete system
A U = (K + gamma M) U = f (Section 1, eq. (positivemaxwell) and
eq. (discretemaxwell)); the bilinear form a(u,v) (Section 2,
eq. (bilinearformposmax)); lowest-order edge elements on a Cartesian mesh
(Section 4, Numerical results); G is the "gradient matrix", the exact null space of the discrete
curl-curl operator (Section 1, the AMS formula).  The paper does not print
the element formulas; the ones below are the textbook Whitney-form ones:
  w_ab = l_a grad l_b - l_b grad l_a,  curl w_ab = 2 grad l_a x grad l_b,
  int_T l_a l_b = |T| (1 + delta_ab) / 20,
with each edge oriented from its lower to its higher global node id.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

# local edges of a tet as pairs of local vertex slots
LOCAL_EDGES = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]


def edge_table(tets):
    """Unique edges as (low id, high id) pairs in lexicographic order, and the
    6 global edge ids of every tet in LOCAL_EDGES order."""
    t = np.asarray(tets, dtype=np.int64)
    pairs = np.stack([t[:, [a for a, _ in LOCAL_EDGES]], t[:, [b for _, b in LOCAL_EDGES]]], axis=-1)
    lo = pairs.min(axis=-1)
    hi = pairs.max(axis=-1)
    nv = int(t.max()) + 1
    key = (lo * nv + hi).ravel()
    uniq, inv = np.unique(key, return_inverse=True)
    edges = np.stack([uniq // nv, uniq % nv], axis=1)
    return edges, inv.reshape(t.shape[0], 6)


def dirichlet_sets(bfaces, dirichlet, edges, n_nodes):
    """Dirichlet nodes = vertices of Dirichlet boundary triangles; Dirichlet
    edges = edges of those triangles (n x E = 0 on Gamma_D, Section 1)."""
    bf = np.asarray(bfaces, dtype=np.int64)[np.asarray(dirichlet) != 0]
    dnode = np.zeros(n_nodes, dtype=bool)
    dnode[bf.ravel()] = True
    nv = n_nodes
    tri_edges = np.concatenate([np.sort(bf[:, [0, 1]], 1), np.sort(bf[:, [0, 2]], 1),
                                np.sort(bf[:, [1, 2]], 1)])
    dkeys = np.unique(tri_edges[:, 0] * nv + tri_edges[:, 1])
    ekeys = edges[:, 0] * nv + edges[:, 1]
    dedge = np.isin(ekeys, dkeys)
    return dnode, dedge


def barycentric_gradients(xyz_tet):
    """Gradients of the 4 barycentric coordinates of one tet and its volume."""
    x0 = xyz_tet[0]
    J = np.stack([xyz_tet[1] - x0, xyz_tet[2] - x0, xyz_tet[3] - x0])  # rows
    # l_k(x) for k=1..3 solves J^T l = x - x0, so grad l_{1..3} = rows of J^{-T}
    Jinv = np.linalg.inv(J)
    g = np.empty((4, 3))
    g[1:] = Jinv.T
    g[0] = -g[1:].sum(axis=0)
    vol = abs(np.linalg.det(J)) / 6.0
    return g, vol


def element_matrices(xyz_tet, gids):
    """Whitney curl-curl (unit mu) and mass (unit eps) matrices of one tet,
    6x6, in LOCAL_EDGES order, each edge oriented low -> high global id."""
    g, vol = barycentric_gradients(xyz_tet)
    ends = []
    for a, b in LOCAL_EDGES:
        ends.append((a, b) if gids[a] < gids[b] else (b, a))
    Ke = np.empty((6, 6))
    Me = np.empty((6, 6))
    for p, (a, b) in enumerate(ends):
        ca = 2.0 * np.cross(g[a], g[b])
        for q, (c, d) in enumerate(ends):
            cc = 2.0 * np.cross(g[c], g[d])
            Ke[p, q] = vol * ca @ cc
            Me[p, q] = vol / 20.0 * ((1 + (a == c)) * g[b] @ g[d] - (1 + (a == d)) * g[b] @ g[c]
                                     - (1 + (b == c)) * g[a] @ g[d] + (1 + (b == d)) * g[a] @ g[c])
    return Ke, Me


def element_matrices_all(xyz, tets):
    """element_matrices() for every tet at once (same formulas, vectorised
    over tets with numpy)."""
    P = xyz[tets]                                     # [T,4,3]
    J = P[:, 1:, :] - P[:, :1, :]                     # rows x_k - x_0
    Jinv = np.linalg.inv(J)
    g = np.empty((tets.shape[0], 4, 3))
    g[:, 1:, :] = np.transpose(Jinv, (0, 2, 1))
    g[:, 0, :] = -g[:, 1:, :].sum(axis=1)
    vol = np.abs(np.linalg.det(J)) / 6.0
    T = tets.shape[0]
    ends = np.empty((T, 6, 2), dtype=np.int64)
    for p, (a, b) in enumerate(LOCAL_EDGES):
        lo_first = tets[:, a] < tets[:, b]
        ends[:, p, 0] = np.where(lo_first, a, b)
        ends[:, p, 1] = np.where(lo_first, b, a)
    ar = np.arange(T)
    Ke = np.empty((T, 6, 6))
    Me = np.empty((T, 6, 6))
    for p in range(6):
        a, b = ends[:, p, 0], ends[:, p, 1]
        ga, gb = g[ar, a], g[ar, b]
        ca = 2.0 * np.cross(ga, gb)
        for q in range(6):
            c, d = ends[:, q, 0], ends[:, q, 1]
            gc, gd = g[ar, c], g[ar, d]
            cc = 2.0 * np.cross(gc, gd)
            Ke[:, p, q] = vol * np.einsum("ij,ij->i", ca, cc)
            dot = lambda u, v: np.einsum("ij,ij->i", u, v)
            Me[:, p, q] = vol / 20.0 * ((1 + (a == c)) * dot(gb, gd) - (1 + (a == d)) * dot(gb, gc)
                                        - (1 + (b == c)) * dot(ga, gd) + (1 + (b == d)) * dot(ga, gc))
    return Ke, Me


class System:
    """The assembled FP64 system over free edges (Section 1, eq. (discretemaxwell))."""

    def __init__(self, mesh, mu, eps, gamma, dirichlet, tets_subset=None):
        xyz = np.asarray(mesh["xyz"], dtype=np.float64)
        tets = np.asarray(mesh["tets"], dtype=np.int64)
        self.mesh = mesh
        self.gamma = float(gamma)
        self.n_nodes = xyz.shape[0]
        self.edges, self.tet_edges = edge_table(tets)
        self.dnode, self.dedge = dirichlet_sets(mesh["bfaces"], dirichlet, self.edges, self.n_nodes)
        self.free_edges = np.nonzero(~self.dedge)[0]
        self.free_nodes = np.nonzero(~self.dnode)[0]
        self.n = self.free_edges.size
        self.p = self.free_nodes.size
        self.edge_to_free = np.full(self.edges.shape[0], -1, np.int64)
        self.edge_to_free[self.free_edges] = np.arange(self.n)
        self.node_to_free = np.full(self.n_nodes, -1, np.int64)
        self.node_to_free[self.free_nodes] = np.arange(self.p)
        # per-tet element matrices (coefficient-free), kept for local Neumann assembly
        T = tets.shape[0]
        self.Ke, self.Me = element_matrices_all(xyz, tets)
        self.mu = np.asarray(mu, dtype=np.float64)
        self.eps = np.asarray(eps, dtype=np.float64)
        self.K = self.assemble_over(np.arange(T), which="K")
        self.M = self.assemble_over(np.arange(T), which="M")
        self.A = (self.K + self.gamma * self.M).tocsr()
        self.G = self.gradient_matrix()

    def assemble_over(self, tet_ids, which="A"):
        """Sum of element contributions of `tet_ids`, restricted to free edges
        (Dirichlet edges eliminated).  which: 'K' (mu^-1 curl-curl), 'M'
        (eps mass) or 'A' (K + gamma M)."""
        tet_ids = np.asarray(tet_ids, dtype=np.int64)
        te = self.edge_to_free[self.tet_edges[tet_ids]]           # [t,6]
        if which == "K":
            loc = self.Ke[tet_ids] / self.mu[tet_ids, None, None]
        elif which == "M":
            loc = self.Me[tet_ids] * self.eps[tet_ids, None, None]
        else:
            loc = (self.Ke[tet_ids] / self.mu[tet_ids, None, None]
                   + self.gamma * self.Me[tet_ids] * self.eps[tet_ids, None, None])
        rows = np.repeat(te, 6, axis=1).ravel()
        cols = np.tile(te, (1, 6)).ravel()
        vals = loc.ravel()
        ok = (rows >= 0) & (cols >= 0)
        m = sp.coo_matrix((vals[ok], (rows[ok], cols[ok])), shape=(self.n, self.n))
        return m.tocsr()

    def gradient_matrix(self):
        """G (free edges x free nodes): G[(a->b), a] = -1, G[(a->b), b] = +1,
        so that grad(phi_k) = sum_e G[e,k] w_e (gradients of H^1 functions that
        vanish on the Dirichlet boundary)."""
        e = self.edges[self.free_edges]
        rows, cols, vals = [], [], []
        for end, sgn in ((0, -1.0), (1, 1.0)):
            c = self.node_to_free[e[:, end]]
            ok = c >= 0
            rows.append(np.nonzero(ok)[0])
            cols.append(c[ok])
            vals.append(np.full(ok.sum(), sgn))
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(self.n, self.p))

    def interpolate(self, field):
        """Edge degrees of freedom of a vector field: the tangential line
        integral along each free edge (5-point Gauss-Legendre)."""
        xyz = self.mesh["xyz"]
        e = self.edges[self.free_edges]
        a, b = xyz[e[:, 0]], xyz[e[:, 1]]
        s, w = np.polynomial.legendre.leggauss(5)
        s = 0.5 * (s + 1.0)
        w = 0.5 * w
        out = np.zeros(self.n)
        for sk, wk in zip(s, w):
            pts = a + sk * (b - a)
            out += wk * np.einsum("ij,ij->i", field(pts), b - a)
        return out


# 4-point degree-2 quadrature on the reference tet (barycentric points, weights sum to 1)
_QA, _QB = 0.5854101966249685, 0.1381966011250105
QUAD_BARY = np.array([[_QA, _QB, _QB, _QB], [_QB, _QA, _QB, _QB], [_QB, _QB, _QA, _QB], [_QB, _QB, _QB, _QA]])
QUAD_W = np.full(4, 0.25)


def _whitney_at(g, ends, bary):
    """Whitney functions of one tet at barycentric point `bary`: [6,3]."""
    return np.array([bary[a] * g[b] - bary[b] * g[a] for a, b in ends])


def _tet_ends(gids):
    return [(a, b) if gids[a] < gids[b] else (b, a) for a, b in LOCAL_EDGES]


def load_vector(system, f):
    """b_e = int_Omega f . w_e over free edges (degree-2 quadrature)."""
    xyz = system.mesh["xyz"]
    tets = system.mesh["tets"]
    out = np.zeros(system.n)
    for t in range(tets.shape[0]):
        P = xyz[tets[t]]
        g, vol = barycentric_gradients(P)
        ends = _tet_ends(tets[t])
        te = system.edge_to_free[system.tet_edges[t]]
        loc = np.zeros(6)
        for lam, w in zip(QUAD_BARY, QUAD_W):
            x = lam @ P
            loc += w * vol * (_whitney_at(g, ends, lam) @ f(x[None, :])[0])
        ok = te >= 0
        out[te[ok]] += loc[ok]
    return out


def l2_errors(system, u, E, curlE):
    """||E - E_h||_L2 and ||curl E - curl E_h||_L2 of the edge-element field
    with free-edge coefficients u (Dirichlet edges carry 0)."""
    xyz = system.mesh["xyz"]
    tets = system.mesh["tets"]
    full = np.zeros(system.edges.shape[0])
    full[system.free_edges] = u
    e0 = e1 = 0.0
    for t in range(tets.shape[0]):
        P = xyz[tets[t]]
        g, vol = barycentric_gradients(P)
        ends = _tet_ends(tets[t])
        c = full[system.tet_edges[t]]
        curl_h = sum(ci * 2.0 * np.cross(g[a], g[b]) for ci, (a, b) in zip(c, ends))
        for lam, w in zip(QUAD_BARY, QUAD_W):
            x = lam @ P
            Eh = c @ _whitney_at(g, ends, lam)
            e0 += w * vol * np.sum((E(x[None, :])[0] - Eh) ** 2)
            e1 += w * vol * np.sum((curlE(x[None, :])[0] - curl_h) ** 2)
    return np.sqrt(e0), np.sqrt(e1)
