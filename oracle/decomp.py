"""Oracle: overlapping decomposition, restriction operators, partition of
unity, local Dirichlet and Neumann matrices, local gradient matrices.

Paper passages (Section 2): Omega = union of overlapping Omega_i conforming
to the mesh; N_i the dofs of Omega_i, R_i the restriction, R_i^T extension by
zero; the algebraic partition of unity sum_i R_i^T D_i R_i = I
(eq. (PoU)); the Dirichlet matrix A_i = R_i A R_i^T (after eq. (AS)); the
Neumann matrix A_i^Neu = the bilinear form integrated over Omega_i only,
with the global boundary conditions kept on the part of the boundary of
Omega_i that lies on the boundary of Omega.  Section 4 (Numerical results): one layer of
elements is added around each non-overlapping subdomain; the paper's
elements are hexes of a Cartesian mesh, so one layer = every hex that
shares a vertex with the subdomain.  G_i = R_i G (Definition "Split
near-kernel coarse space").

Readings where the paper is silent:
  * the partition of unity: with l overlap layers, chi_i is 1 at the nodes
    of the original (non-overlapping) cells of subdomain i, 1 - d/l at nodes
    first reached by the d-th added layer (0 on the outer boundary of
    Omega_i); its edge value is the mean of the two end values, and
    D_i = chi_i / sum_j chi_j.  This is the usual "smooth" Schwarz PoU.  The
    multiplicity PoU D_i = 1/m_e (also provided) makes the columns
    R_i^T D_i G_i linearly dependent wherever a node's whole edge star lies in
    the same overlap, so Z would not be a basis and E would be singular;
  * G_i keeps the columns of the free nodes touched by N_i; in every
    connected component of that node set that reaches no Dirichlet node the
    columns sum to zero, so the lowest-numbered node of each such component
    is dropped (G_i must have full column rank for E and S_i to be SPD).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.csgraph as csg


def box_partition(mesh, p):
    """Non-overlapping partition of the cells (hexes) into a px*py*pz grid of
    boxes by cell centroid."""
    xyz = mesh["xyz"]
    tets = mesh["tets"]
    hot = mesh["hex_of_tet"]
    H = int(hot.max()) + 1
    cent = np.zeros((H, 3))
    np.add.at(cent, hot, xyz[tets].mean(axis=1))
    cent /= np.bincount(hot, minlength=H)[:, None]
    lo = xyz.min(axis=0)
    hi = xyz.max(axis=0)
    idx = []
    for a in range(3):
        k = np.floor((cent[:, a] - lo[a]) / (hi[a] - lo[a]) * p[a]).astype(np.int64)
        idx.append(np.clip(k, 0, p[a] - 1))
    return idx[0] + p[0] * (idx[1] + p[1] * idx[2])


def cell_centroids(mesh):
    xyz = mesh["xyz"]
    hot = mesh["hex_of_tet"]
    H = int(hot.max()) + 1
    cent = np.zeros((H, 3))
    np.add.at(cent, hot, xyz[mesh["tets"]].mean(axis=1))
    return cent / np.bincount(hot, minlength=H)[:, None]


def rcb_partition(mesh, nparts, jitter):
    """Recursive coordinate bisection of the cells into `nparts` parts.

    A node holding k parts and a set of cells splits along the axis of the
    largest centroid extent (lowest axis on ties), cells ordered by
    (centroid coordinate, cell id); the first
      clip(round(n * floor(k/2)/k * (1 + jitter)), floor(k/2), n - ceil(k/2))
    cells get floor(k/2) parts, the rest ceil(k/2).  `jitter` holds one value
    per internal node of the bisection tree, consumed in preorder (root, left
    subtree, right subtree); part ids are assigned left to right."""
    cent = cell_centroids(mesh)
    part = np.empty(cent.shape[0], dtype=np.int64)
    state = {"j": 0, "next_part": 0}

    def rec(cells, k):
        if k == 1:
            part[cells] = state["next_part"]
            state["next_part"] += 1
            return
        d = float(jitter[state["j"]])
        state["j"] += 1
        c = cent[cells]
        ext = c.max(axis=0) - c.min(axis=0)
        axis = int(np.argmax(ext))
        order = np.lexsort((cells, c[:, axis]))
        cells = cells[order]
        kl, kr = k // 2, k - k // 2
        n = cells.size
        nl = int(np.floor(n * kl / k * (1.0 + d) + 0.5))
        nl = min(max(nl, kl), n - kr)
        rec(cells[:nl], kl)
        rec(cells[nl:], kr)

    rec(np.arange(cent.shape[0]), int(nparts))
    return part


def cell_adjacency(mesh):
    """Cells sharing at least one vertex (sparse boolean, symmetric)."""
    hot = mesh["hex_of_tet"]
    H = int(hot.max()) + 1
    tets = mesh["tets"]
    nv = mesh["xyz"].shape[0]
    rows = np.repeat(hot, 4)
    cols = tets.ravel()
    C = sp.csr_matrix((np.ones(rows.size), (rows, cols)), shape=(H, nv))
    C.data[:] = 1.0
    adj = (C @ C.T).tocsr()
    adj.data[:] = 1.0
    return adj


class Decomposition:
    """Overlapping subdomains and their local operators (Section 2)."""

    def __init__(self, system, part_of_cell, overlap, pou="smooth"):
        mesh = system.mesh
        self.sys = system
        hot = np.asarray(mesh["hex_of_tet"], dtype=np.int64)
        H = int(hot.max()) + 1
        part_of_cell = np.asarray(part_of_cell, dtype=np.int64)
        self.N = int(part_of_cell.max()) + 1
        adj = cell_adjacency(mesh)
        tets_of_cell = [[] for _ in range(H)]
        for t, c in enumerate(hot):
            tets_of_cell[c].append(t)
        self.overlap = int(overlap)
        tets_all = np.asarray(mesh["tets"], dtype=np.int64)
        nn = system.n_nodes
        free_e = system.edges[system.free_edges]
        self.cells, self.tets, self.dofs, self.chi = [], [], [], []
        for i in range(self.N):
            inside = part_of_cell == i
            level = np.where(inside, 0, -1)
            for d in range(1, overlap + 1):
                grown = inside | (adj @ inside.astype(np.float64) > 0)
                level[grown & ~inside] = d
                inside = grown
            cells = np.nonzero(inside)[0]
            tets = np.sort(np.concatenate([tets_of_cell[c] for c in cells]))
            e = system.edge_to_free[system.tet_edges[tets]].ravel()
            dofs = np.unique(e[e >= 0])
            # nodal level d(v) = lowest level of a cell of Omega_i holding v
            dv = np.full(nn, overlap + 1, dtype=np.int64)
            np.minimum.at(dv, tets_all[tets].ravel(), np.repeat(level[hot[tets]], 4))
            chi_node = 1.0 - dv / max(overlap, 1) if overlap else (dv == 0).astype(float)
            ends = free_e[dofs]
            self.chi.append(0.5 * (chi_node[ends[:, 0]] + chi_node[ends[:, 1]]))
            self.cells.append(cells)
            self.tets.append(tets)
            self.dofs.append(dofs)
        # multiplicity of each free edge
        self.mult = np.zeros(system.n, dtype=np.int64)
        for d in self.dofs:
            self.mult[d] += 1
        if pou == "multiplicity":
            self.D = [1.0 / self.mult[d] for d in self.dofs]
        else:
            tot = np.zeros(system.n)
            for d, c in zip(self.dofs, self.chi):
                tot[d] += c
            self.D = [c / tot[d] for d, c in zip(self.dofs, self.chi)]

    # R_i as a sparse n_i x n matrix
    def R(self, i):
        d = self.dofs[i]
        return sp.csr_matrix((np.ones(d.size), (np.arange(d.size), d)), shape=(d.size, self.sys.n))

    def A_dir(self, i):
        """A_i = R_i A R_i^T (Section 2, after eq. (AS))."""
        d = self.dofs[i]
        return self.sys.A[d][:, d].tocsr()

    def A_neu(self, i):
        """A_i^Neu: the bilinear form assembled over the tets of Omega_i only,
        restricted to N_i (Section 2)."""
        d = self.dofs[i]
        full = self.sys.assemble_over(self.tets[i], which="A")
        return full[d][:, d].tocsr()

    def G_local(self, i):
        """G_i = R_i G restricted to its non-zero columns, minus the lowest
        node of every floating component.  Returns (G_i sparse n_i x p_i,
        global free-node ids of the kept columns, number dropped)."""
        d = self.dofs[i]
        Gi = self.sys.G[d].tocsc()
        nz = np.nonzero(np.diff(Gi.indptr) > 0)[0]
        Gi = Gi[:, nz]
        # connected components over local free nodes via edges with two free ends
        Gr = Gi.tocsr()
        cnt = np.diff(Gr.indptr)
        both = np.nonzero(cnt == 2)[0]
        one = np.nonzero(cnt == 1)[0]
        a = Gr.indices[Gr.indptr[both]]
        b = Gr.indices[Gr.indptr[both] + 1]
        m = nz.size
        g = sp.coo_matrix((np.ones(both.size), (a, b)), shape=(m, m))
        ncomp, lab = csg.connected_components(g, directed=False)
        anchored = np.zeros(ncomp, dtype=bool)
        anchored[lab[Gr.indices[Gr.indptr[one]]]] = True   # edge to a Dirichlet node
        drop = []
        for c in range(ncomp):
            if not anchored[c]:
                drop.append(np.nonzero(lab == c)[0].min())
        keep = np.setdiff1d(np.arange(m), np.asarray(drop, dtype=np.int64))
        return Gi[:, keep].tocsr(), nz[keep], len(drop)


def partition_cells(workload):
    """Non-overlapping cell partition from a workload's partition options."""
    opt = workload.partition
    if opt["kind"] == "box":
        return box_partition(workload.mesh, opt["p"])
    if opt["kind"] == "rcb":
        return rcb_partition(workload.mesh, opt["nparts"], opt["jitter"])
    if opt["kind"] == "explicit":
        return np.asarray(opt["part"], dtype=np.int64)
    raise ValueError(opt["kind"])
