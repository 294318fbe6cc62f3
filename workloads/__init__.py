"""Seeded synthetic workloads: meshes, coefficient fields, right-hand sides.

This module only *describes inputs*.  It holds none of the preconditioner's
arithmetic (no element matrices, no edges, no decomposition): it builds the
tetrahedral mesh of a Cartesian hex grid, tags its boundary triangles, draws
the coefficient fields mu / eps and the right-hand side, and states the
decomposition options of each workload.  Both the CPU oracle and the HIP
library read what it returns.

Mesh conventions (the paper only says "Cartesian mesh", Section 4 "Numerical results"):
  * node (i, j, k) of an X*Y*Z hex grid has id i + (X+1)*(j + (Y+1)*k), with
    coordinates h*(i, j, k); nodes used by no kept hex are dropped and the
    remaining ids compacted in increasing order;
  * hex (hx, hy, hz) has id hx + X*(hy + Y*hz) before removal of hole hexes;
  * each hex is split into 6 Kuhn tets [c000, c000+e_a, c000+e_a+e_b, c111],
    one per permutation (a, b, c) of the axes, in itertools order;
  * boundary triangles are the halves of hex faces that have no kept
    neighbour; a face is cut along the diagonal from its lowest to its
    highest corner, which is the diagonal the Kuhn split puts on it.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np

# Boundary-face tags: 0..5 = outer faces -x, +x, -y, +y, -z, +z; 6 = hole wall.
TAG_HOLE = 6

_PERMS = list(itertools.permutations((0, 1, 2)))


def hex_box_mesh(dims, h=None, removed=None):
    """Tet mesh of an X*Y*Z hex grid with optional removed (hole) hexes.

    Returns a dict with xyz f64[V,3], tets i32[T,4], hex_of_tet i32[T],
    hex_ijk i32[H,3] (grid coordinates of kept hexes), bfaces i32[F,3],
    bface_tag i8[F] and dims / h.
    """
    X, Y, Z = (int(d) for d in dims)
    if h is None:
        h = 1.0 / min(X, Y, Z)
    keep = np.ones((X, Y, Z), dtype=bool)
    if removed is not None:
        keep &= ~np.asarray(removed, dtype=bool)
    hx, hy, hz = np.nonzero(keep.transpose(2, 1, 0))[::-1]  # hex-id order
    # np.nonzero on the (Z,Y,X) transpose enumerates hexes with x fastest
    hex_ijk = np.stack([hx, hy, hz], axis=1).astype(np.int64)
    H = hex_ijk.shape[0]

    def nid(i, j, k):
        return i + (X + 1) * (j + (Y + 1) * k)

    unit = np.eye(3, dtype=np.int64)
    tets = np.empty((H, 6, 4), dtype=np.int64)
    for p, (a, b, _c) in enumerate(_PERMS):
        corners = [np.zeros(3, np.int64), unit[a], unit[a] + unit[b], np.ones(3, np.int64)]
        for v, off in enumerate(corners):
            q = hex_ijk + off
            tets[:, p, v] = nid(q[:, 0], q[:, 1], q[:, 2])
    tets = tets.reshape(H * 6, 4)
    hex_of_tet = np.repeat(np.arange(H, dtype=np.int64), 6)

    # boundary faces: hex faces whose neighbour is outside the grid or removed
    padded = np.zeros((X + 2, Y + 2, Z + 2), dtype=bool)
    padded[1:-1, 1:-1, 1:-1] = keep
    tris, tags = [], []
    for f in range(3):
        u, v = [a for a in range(3) if a != f]
        for side in (0, 1):
            nb = hex_ijk.copy()
            nb[:, f] += 1 if side else -1
            outside = (nb[:, f] < 0) | (nb[:, f] >= (X, Y, Z)[f])
            nb_keep = padded[nb[:, 0] + 1, nb[:, 1] + 1, nb[:, 2] + 1]
            sel = ~nb_keep
            if not sel.any():
                continue
            base = hex_ijk[sel].copy()
            base[:, f] += side
            p0 = base
            pu = base + unit[u]
            pv = base + unit[v]
            puv = base + unit[u] + unit[v]
            ids = [nid(q[:, 0], q[:, 1], q[:, 2]) for q in (p0, pu, pv, puv)]
            t1 = np.stack([ids[0], ids[1], ids[3]], axis=1)
            t2 = np.stack([ids[0], ids[2], ids[3]], axis=1)
            tag = np.where(outside[sel], 2 * f + side, TAG_HOLE).astype(np.int8)
            tris += [t1, t2]
            tags += [tag, tag]
    bfaces = np.concatenate(tris, axis=0) if tris else np.zeros((0, 3), np.int64)
    bface_tag = np.concatenate(tags) if tags else np.zeros(0, np.int8)

    # compact node ids (drop nodes that belong to removed hexes only)
    used = np.unique(tets)
    remap = np.full((X + 1) * (Y + 1) * (Z + 1), -1, dtype=np.int64)
    remap[used] = np.arange(used.size)
    gi = used % (X + 1)
    gj = (used // (X + 1)) % (Y + 1)
    gk = used // ((X + 1) * (Y + 1))
    xyz = h * np.stack([gi, gj, gk], axis=1).astype(np.float64)
    return dict(
        xyz=np.ascontiguousarray(xyz),
        tets=np.ascontiguousarray(remap[tets].astype(np.int32)),
        hex_of_tet=hex_of_tet.astype(np.int32),
        hex_ijk=hex_ijk.astype(np.int32),
        bfaces=np.ascontiguousarray(remap[bfaces].astype(np.int32)),
        bface_tag=bface_tag,
        dims=(X, Y, Z),
        h=float(h),
    )


def dirichlet_flags(bface_tag, rule="all"):
    """1 = Dirichlet (n x E = 0), 0 = natural (Neumann) condition, per triangle.

    rule: 'all' (every boundary face), 'outer' (outer faces Dirichlet, hole
    walls Neumann), 'mixed' (Neumann on the two opposing lateral faces -y/+y,
    Dirichlet elsewhere, as in the paper's mixed beam case), 'none'.
    """
    t = np.asarray(bface_tag)
    if rule == "all":
        d = np.ones(t.shape, bool)
    elif rule == "outer":
        d = t != TAG_HOLE
    elif rule == "mixed":
        d = (t != 2) & (t != 3)
    elif rule == "none":
        d = np.zeros(t.shape, bool)
    else:
        raise ValueError(f"unknown boundary rule {rule!r}")
    return d.astype(np.int8)


def rhs(n, rng):
    """Right-hand side with i.i.d. N(0,1) entries in free-edge order."""
    return rng.standard_normal(int(n))


# ---------------------------------------------------------------- coefficients

def channel_mu(dims, rng, frac=0.10, high=1e4, width=2):
    """mu = `high` on seeded random axis-aligned straight channels of a
    width x width hex cross-section until at least `frac` of the hexes are
    covered, 1 elsewhere.  Returns a (X,Y,Z) array."""
    X, Y, Z = dims
    mu = np.ones((X, Y, Z))
    target = frac * X * Y * Z
    while (mu > 1).sum() < target:
        axis = int(rng.integers(0, 3))
        others = [a for a in range(3) if a != axis]
        o = [int(rng.integers(0, dims[a] - width + 1)) for a in others]
        sl = [slice(None)] * 3
        for a, oo in zip(others, o):
            sl[a] = slice(oo, oo + width)
        mu[tuple(sl)] = high
    return mu


def slab_mu(dims, nslab=8, lo=1.0, hi=1e3):
    """Alternating mu = lo, hi, lo, ... in `nslab` equal slabs along x."""
    X, Y, Z = dims
    mu = np.empty((X, Y, Z))
    w = X // nslab
    for s in range(nslab):
        mu[s * w:(s + 1) * w] = lo if s % 2 == 0 else hi
    return mu


def per_hex(field3d, mesh):
    """Gather a (X,Y,Z) per-hex field onto the kept hexes, then onto tets."""
    ijk = mesh["hex_ijk"]
    per_h = field3d[ijk[:, 0], ijk[:, 1], ijk[:, 2]]
    return np.ascontiguousarray(per_h[mesh["hex_of_tet"]].astype(np.float64))


# ---------------------------------------------------------------- workloads

@dataclass
class Workload:
    """One synthetic problem: mesh + coefficients + decomposition options."""
    name: str
    mesh: dict
    mu: np.ndarray           # f64[T]
    eps: np.ndarray          # f64[T]
    gamma: float
    dirichlet: np.ndarray    # i8[F]
    partition: dict          # {"kind": "box", "p": (px,py,pz)} | {"kind": "rcb", ...} | {"kind": "explicit", "part": i32[H]}
    overlap: int
    tau: float = 10.0
    nev_max: int = 20
    seed: int = 0
    extra: dict = field(default_factory=dict)
    describe: str = ""       # one-line statement of the recipe (mesh, coefficients, decomposition)

    def rhs(self, n):
        ss = np.random.SeedSequence(self.seed).spawn(4)
        return rhs(n, np.random.default_rng(ss[1]))

    def start_rng(self):
        """Stream for random LOBPCG start blocks."""
        ss = np.random.SeedSequence(self.seed).spawn(4)
        return np.random.default_rng(ss[3])


def paper_beam(N, gamma=1e-3, bc="all", layers=None, alt=1.0, cells=16):
    """The paper's beam (Section 4, Numerical results): N/2 x 1 x 1 with
    h = 1 / cells (the paper: 16), i.e. (cells N / 2) x cells x cells hexes,
    N strip subdomains along its length, one overlap layer, tau = 10.
    bc: "all" (Dirichlet on every face) or "mixed" (Neumann on the two
    opposing lateral faces -y / +y).  layers: None (mu = eps = 1), "eps" or
    "mu": eight alternating layers along the length, the coefficient 1 in
    the first and `alt` in the second (Tables 7 and 8 of the paper's
    heterogeneity study); gamma as in its gamma sweep (Table 5)."""
    X = cells * N // 2
    if X % 8 and layers:
        raise ValueError("eight layers need a length divisible by 8 cells")
    dims = (X, cells, cells)
    mesh = hex_box_mesh(dims, h=1.0 / cells)
    T = mesh["tets"].shape[0]
    mu, eps = np.ones(T), np.ones(T)
    if layers == "mu":
        mu = per_hex(slab_mu(dims, nslab=8, lo=1.0, hi=alt), mesh)
    elif layers == "eps":
        eps = per_hex(slab_mu(dims, nslab=8, lo=1.0, hi=alt), mesh)
    elif layers is not None:
        raise ValueError(f"unknown layers {layers!r}")
    name = f"paper_beam{N}_h{cells}_{bc}" + (f"_{layers}{alt:g}" if layers else "") + f"_g{gamma:g}"
    desc = (f"beam {X}x{cells}x{cells} hexes x 6 tets, h = 1/{cells}, {N} strips, overlap 1, gamma = {gamma:g}, "
            + ("all-Dirichlet" if bc == "all" else "Neumann on -y/+y, Dirichlet elsewhere")
            + (f", {layers} alternating 1 / {alt:g} in 8 layers" if layers else ", mu = eps = 1"))
    return Workload(name, mesh, mu, eps, float(gamma), dirichlet_flags(mesh["bface_tag"], bc),
                    {"kind": "box", "p": (N, 1, 1)}, 1, seed=4000 + N, describe=desc)


def rcb_jitter(nparts, rng, spread=0.3):
    """Per-split size jitter for recursive coordinate bisection, one value per
    internal node of the bisection tree in preorder (nparts-1 values).  The
    spread is divided by the tree depth so that compounded part sizes stay
    within roughly +-spread of the mean."""
    depth = max(1, int(np.ceil(np.log2(max(nparts, 2)))))
    return rng.uniform(-spread, spread, size=max(nparts - 1, 0)) / depth


def make(cfg, family=0, **over):
    """Build workload `cfg` (1 - 5, or a small named test case).

    family > 0: another instance of the same recipe, its random draws taken
    from the streams SeedSequence([seed, family]) instead of SeedSequence(seed):
    new channels (config 2, "small_channels"), new lognormal fields and
    bisection jitter (config 3), new inclusions and gamma (config 4), new
    bisection jitter (config 5, whose slab
    coefficients are fixed, so the subdomains change shape and position).
    Used to train the learned warm start on instances disjoint from the
    measured one (family 0)."""
    def stream(seed):
        return np.random.SeedSequence([seed, family] if family else seed).spawn(4)
    if cfg == 1:
        dims = (8, 8, 8)
        mesh = hex_box_mesh(dims)
        T = mesh["tets"].shape[0]
        w = Workload("cube8_homog", mesh, np.ones(T), np.ones(T), 1e-2,
                     dirichlet_flags(mesh["bface_tag"], "all"),
                     {"kind": "box", "p": (2, 2, 2)}, 1, seed=1001,
                     describe="unit cube 8^3 hexes x 6 tets (3,072), mu = eps = 1, gamma = 1e-2, "
                              "all-Dirichlet, 2x2x2 boxes, overlap 1")
    elif cfg == 2:
        dims = (24, 24, 24)
        mesh = hex_box_mesh(dims)
        ss = stream(1002)
        mu = per_hex(channel_mu(dims, np.random.default_rng(ss[0])), mesh)
        T = mesh["tets"].shape[0]
        w = Workload("cube24_channels", mesh, mu, np.ones(T), 1e-4,
                     dirichlet_flags(mesh["bface_tag"], "all"),
                     {"kind": "box", "p": (4, 4, 4)}, 2, seed=1002,
                     describe="24^3 hexes x 6 tets (82,944), mu in {1, 1e4} on random 2x2-hex channels "
                              ">= 10%, eps = 1, gamma = 1e-4, all-Dirichlet, 4x4x4 boxes, overlap 2")
    elif cfg == 3:
        dims = (32, 32, 32)
        removed = np.zeros(dims, bool)
        removed[12:20, 12:20, :] = True
        mesh = hex_box_mesh(dims, removed=removed)
        ss = stream(1003)
        r = np.random.default_rng(ss[0])
        H = mesh["hex_ijk"].shape[0]
        lmu = r.normal(0.0, 2.0, size=H)
        leps = r.normal(0.0, 2.0, size=H)
        mu = np.exp(lmu)[mesh["hex_of_tet"]]
        eps = np.exp(leps)[mesh["hex_of_tet"]]
        jit = rcb_jitter(125, np.random.default_rng(ss[2]))
        w = Workload("cube32_hole_lognormal", mesh, mu, eps, 1e-3,
                     dirichlet_flags(mesh["bface_tag"], "outer"),
                     {"kind": "rcb", "nparts": 125, "jitter": jit}, 1, seed=1003,
                     describe="32^3 hexes minus a central 8x8x32 through-hole (184,320 tets), lognormal "
                              "mu, eps (sigma 2), gamma = 1e-3, Dirichlet outside / Neumann on the hole, "
                              "RCB 125 parts (+-30% jitter), overlap 1")
    elif cfg == 4:
        # Training instances of the learned warm start: subdomains of 12^3 cells (11^3-hex boxes
        # plus one overlap layer) of a 22^3 cube, mu = 10^U(0, 5) on 4..8 seeded random box
        # inclusions of 2..6 cells per side (1 elsewhere), eps = 1, gamma = 10^U(-6, 0).
        dims = (22, 22, 22)
        mesh = hex_box_mesh(dims)
        ss = stream(1004)
        r = np.random.default_rng(ss[0])
        mu3 = np.ones(dims)
        for _ in range(int(r.integers(4, 9))):
            size = r.integers(2, 7, size=3)
            lo = [int(r.integers(0, dims[a] - size[a] + 1)) for a in range(3)]
            mu3[lo[0]:lo[0] + size[0], lo[1]:lo[1] + size[1], lo[2]:lo[2] + size[2]] = 10.0 ** r.uniform(0, 5)
        gamma = 10.0 ** r.uniform(-6, 0)
        T = mesh["tets"].shape[0]
        w = Workload("cube22_inclusions", mesh, per_hex(mu3, mesh), np.ones(T), gamma,
                     dirichlet_flags(mesh["bface_tag"], "all"),
                     {"kind": "box", "p": (2, 2, 2)}, 1, seed=1004,
                     describe=f"22^3 hexes x 6 tets (63,888), mu = 10^U(0,5) on 4-8 random box inclusions, eps = 1, "
                              f"gamma = {gamma:.3g} (10^U(-6,0)), all-Dirichlet, 2x2x2 boxes (12^3 cells with "
                              "the overlap layer), overlap 1")
    elif cfg == 5:
        dims = (128, 16, 16)
        mesh = hex_box_mesh(dims, h=1.0 / 16)
        ss = stream(1005)
        mu = per_hex(slab_mu(dims), mesh)
        T = mesh["tets"].shape[0]
        jit = rcb_jitter(256, np.random.default_rng(ss[2]))
        w = Workload("beam128_slabs", mesh, mu, np.ones(T), 1e-6,
                     dirichlet_flags(mesh["bface_tag"], "all"),
                     {"kind": "rcb", "nparts": 256, "jitter": jit}, 1, seed=1005,
                     describe="beam 128x16x16 hexes x 6 tets (196,608), h = 1/16, mu alternating 1 / 1e3 "
                              "in 8 slabs along x, eps = 1, gamma = 1e-6, all-Dirichlet, RCB 256 parts "
                              "(+-30% jitter), overlap 1")
    elif cfg == "cube24_homog":
        # The 24^3 cube of config 2 with the homogeneous coefficients and gamma of config 1: the
        # same subdomain sizes (n_i 3,584 .. 7,930), local matrices well enough conditioned for
        # FP32 factors (measures the FP32 local factorisation).
        dims = (24, 24, 24)
        mesh = hex_box_mesh(dims)
        T = mesh["tets"].shape[0]
        w = Workload("cube24_homog", mesh, np.ones(T), np.ones(T), 1e-2,
                     dirichlet_flags(mesh["bface_tag"], "all"),
                     {"kind": "box", "p": (4, 4, 4)}, 2, seed=2005,
                     describe="24^3 hexes x 6 tets (82,944), mu = eps = 1, gamma = 1e-2, all-Dirichlet, "
                              "4x4x4 boxes, overlap 2")
    elif isinstance(cfg, str) and cfg.startswith("beam") and cfg[4:].isdigit():
        # The paper's weak-scaling beam (Section 4 "Numerical results", influence of the geometry):
        # N/2 x 1 x 1 with h = 1/16 (8N x 16 x 16 hexes), N strip subdomains
        # along the length, one overlap layer, mu = eps = 1, gamma = 1e-3,
        # Dirichlet on all faces (rule "mixed": Neumann on two opposing
        # lateral faces instead).
        N = int(cfg[4:])
        dims = (8 * N, 16, 16)
        mesh = hex_box_mesh(dims, h=1.0 / 16)
        T = mesh["tets"].shape[0]
        w = Workload(f"beam{N}_strips", mesh, np.ones(T), np.ones(T), 1e-3,
                     dirichlet_flags(mesh["bface_tag"], "all"),
                     {"kind": "box", "p": (N, 1, 1)}, 1, seed=3000 + N)
    elif cfg == "small_channels":
        # A small heterogeneous case whose GenEO space is not empty.
        dims = (8, 8, 8)
        mesh = hex_box_mesh(dims)
        ss = stream(2001)
        mu = per_hex(channel_mu(dims, np.random.default_rng(ss[0]), frac=0.15), mesh)
        T = mesh["tets"].shape[0]
        w = Workload("cube8_channels", mesh, mu, np.ones(T), 1e-4,
                     dirichlet_flags(mesh["bface_tag"], "all"),
                     {"kind": "box", "p": (2, 2, 2)}, 1, seed=2001)
    elif cfg == "small_mixed":
        # Small beam with Neumann lateral faces and floating-free subdomains.
        dims = (12, 4, 4)
        mesh = hex_box_mesh(dims, h=0.25)
        T = mesh["tets"].shape[0]
        mu = per_hex(slab_mu(dims, nslab=4, hi=1e3), mesh)
        w = Workload("beam12_mixed", mesh, mu, np.ones(T), 1e-3,
                     dirichlet_flags(mesh["bface_tag"], "mixed"),
                     {"kind": "box", "p": (3, 1, 1)}, 1, seed=2002)
    elif cfg == "small_floating":
        # 6^3 interior subdomain is floating (touches no Dirichlet face).
        dims = (9, 9, 9)
        mesh = hex_box_mesh(dims)
        T = mesh["tets"].shape[0]
        ss = np.random.SeedSequence(2003).spawn(4)
        mu = per_hex(channel_mu(dims, np.random.default_rng(ss[0]), frac=0.1), mesh)
        w = Workload("cube9_floating", mesh, mu, np.ones(T), 1e-3,
                     dirichlet_flags(mesh["bface_tag"], "all"),
                     {"kind": "box", "p": (3, 3, 3)}, 1, seed=2003)
    elif cfg == "small_hole":
        dims = (8, 8, 6)
        removed = np.zeros(dims, bool)
        removed[3:5, 3:5, :] = True
        mesh = hex_box_mesh(dims, removed=removed)
        ss = np.random.SeedSequence(2004).spawn(4)
        r = np.random.default_rng(ss[0])
        H = mesh["hex_ijk"].shape[0]
        mu = np.exp(r.normal(0, 2.0, H))[mesh["hex_of_tet"]]
        eps = np.exp(r.normal(0, 2.0, H))[mesh["hex_of_tet"]]
        jit = rcb_jitter(7, np.random.default_rng(ss[2]))
        w = Workload("cube8_hole_rcb", mesh, mu, eps, 1e-3,
                     dirichlet_flags(mesh["bface_tag"], "outer"),
                     {"kind": "rcb", "nparts": 7, "jitter": jit}, 1, seed=2004)
    else:
        raise ValueError(f"unknown workload {cfg!r}")
    if family:
        if cfg not in (2, 3, 4, 5, "small_channels"):
            raise ValueError(f"no instance family for workload {cfg!r}")
        w.name = f"{w.name}#{family}"
    for k, v in over.items():
        setattr(w, k, v)
    return w
