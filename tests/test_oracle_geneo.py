"""Pins of the oracle's decomposition, GEVP, coarse space and two-level
preconditioner (no GPU)."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import workloads as W
from oracle import decomp, fem, geneo


def _case(dims, p, overlap=1, rule="all", gamma=1e-3, contrast=1e3, seed=0, removed=None):
    mesh = W.hex_box_mesh(dims, removed=removed)
    T = mesh["tets"].shape[0]
    rng = np.random.default_rng(seed)
    H = mesh["hex_ijk"].shape[0]
    mu_h = np.where(rng.random(H) < 0.2, contrast, 1.0)
    s = fem.System(mesh, mu_h[mesh["hex_of_tet"]], np.ones(T), gamma,
                   W.dirichlet_flags(mesh["bface_tag"], rule))
    part = decomp.box_partition(mesh, p)
    return s, decomp.Decomposition(s, part, overlap)


@pytest.fixture(scope="module")
def tiny():
    return _case((4, 4, 4), (2, 2, 1))


@pytest.fixture(scope="module")
def floating():
    # 3x3x3 boxes of a 6^3 cube: the centre subdomain touches no boundary
    return _case((6, 6, 6), (3, 3, 3), gamma=1e-2, contrast=1e2, seed=1)


def test_partition_of_unity(tiny, floating):
    """sum_i R_i^T D_i R_i = I (Section 2, eq. (PoU))."""
    for s, dec in (tiny, floating):
        I = sum(dec.R(i).T @ sp.diags(dec.D[i]) @ dec.R(i) for i in range(dec.N))
        assert abs(I - sp.eye(s.n)).max() < 1e-14
        assert all((d >= 0).all() for d in dec.D)


def test_dirichlet_and_neumann_local_matrices(tiny):
    """A_i = R_i A R_i^T; A_i^Neu <= A_i (the Dirichlet matrix adds the
    contributions of the outside elements touching the interface), both SPD
    because gamma > 0 (Section 2)."""
    s, dec = tiny
    for i in range(dec.N):
        Ri = dec.R(i)
        Ai = dec.A_dir(i).toarray()
        assert np.allclose(Ai, (Ri @ s.A @ Ri.T).toarray())
        Neu = dec.A_neu(i).toarray()
        assert np.linalg.eigvalsh(Neu).min() > 0
        assert np.linalg.eigvalsh(Ai - Neu).min() > -1e-12 * abs(Ai).max()


def test_xi_projection_identities(tiny, floating):
    """xi_0i is the b_i-orthogonal projection on span(G_i) (Section 2):
    xi^2 = xi, xi G_i = G_i, A_i xi symmetric."""
    for s, dec in (tiny, floating):
        for i in range(dec.N):
            Ai = dec.A_dir(i).toarray()
            Gi, _, _ = dec.G_local(i)
            X = geneo.xi_projection(Ai, Gi)
            assert np.allclose(X @ X, X, atol=1e-9)
            assert np.allclose(X @ Gi.toarray(), Gi.toarray(), atol=1e-9)
            AX = Ai @ X
            assert np.allclose(AX, AX.T, atol=1e-9 * abs(AX).max())


def test_floating_component_dropped(floating):
    """The centre subdomain reaches no Dirichlet node: its G_i loses exactly
    one column, and what remains has full column rank."""
    s, dec = floating
    drops = [dec.G_local(i)[2] for i in range(dec.N)]
    assert sum(drops) == 1 and drops[13] == 1
    for i in range(dec.N):
        Gi = dec.G_local(i)[0].toarray()
        assert np.linalg.matrix_rank(Gi) == Gi.shape[1]


def test_gevp_against_brute_force(tiny):
    """The filtered GEVP (Section 3.2, eq. (eigAtildeBAS)): its eigenvalues
    equal those of the non-symmetric matrix B^-1 Atilde (numpy.linalg.eig),
    all are >= 0, G_i lies in the lambda = 0 eigenspace, and eigenvectors
    with lambda > 0 are B-orthogonal to span(G_i)."""
    s, dec = tiny
    for i in range(dec.N):
        Ai = dec.A_dir(i).toarray()
        Neu = dec.A_neu(i).toarray()
        Gi, _, _ = dec.G_local(i)
        lam, V, sel = geneo.gevp(Ai, Neu, dec.D[i], Gi, tau=10.0, nev_max=0)
        At, B = geneo.filtered_pencil(Ai, Neu, dec.D[i], Gi)
        ev = np.sort(np.linalg.eig(np.linalg.solve(B, At))[0].real)[::-1]
        assert np.allclose(lam[:10], ev[:10], rtol=1e-8)
        assert lam.min() > -1e-10 * lam.max()
        assert np.allclose(At @ Gi.toarray(), 0, atol=1e-9 * abs(At).max())
        pos = lam > 1e-8 * lam[0]
        Gd = Gi.toarray()
        assert abs(Gd.T @ B @ V[:, pos]).max() < 1e-8 * np.sqrt(abs(B).max())


def test_gevp_lemma_bound(tiny):
    """Lemma (GEVP bound, Section 3.2): for all U,
    (A_i D (I-xi)(I-pi)U, D (I-xi)(I-pi)U) <= tau (A_i^Neu U, U), where pi
    projects on the eigenvectors with lambda > tau (no cap)."""
    s, dec = tiny
    rng = np.random.default_rng(5)
    tau = 2.0   # small tau so that the space being removed is not empty
    for i in range(dec.N):
        Ai = dec.A_dir(i).toarray()
        Neu = dec.A_neu(i).toarray()
        Gi, _, _ = dec.G_local(i)
        lam, V, sel = geneo.gevp(Ai, Neu, dec.D[i], Gi, tau=tau, nev_max=0)
        Vt = V[:, :sel]
        xi = geneo.xi_projection(Ai, Gi)
        Q = np.eye(Ai.shape[0]) - xi
        for _ in range(5):
            U = rng.normal(size=Ai.shape[0])
            U1 = U - Vt @ (Vt.T @ (Neu @ U))      # (I - pi) U, pi B-orthogonal
            w = dec.D[i] * (Q @ U1)
            assert w @ Ai @ w <= tau * (U @ Neu @ U) * (1 + 1e-9)


def test_classical_pencil_has_more_large_eigenvalues(tiny):
    """Section 3.2, remark: the classical pencil D A D V = lambda A^Neu V has
    many more eigenvalues above tau than the filtered one."""
    s, dec = tiny
    i = 0
    Ai = dec.A_dir(i).toarray()
    Neu = dec.A_neu(i).toarray()
    Gi, _, _ = dec.G_local(i)
    lf, _, sf = geneo.gevp(Ai, Neu, dec.D[i], Gi, tau=10.0, nev_max=0)
    lc, _, sc = geneo.gevp(Ai, Neu, dec.D[i], Gi, tau=10.0, nev_max=0, classical=True)
    assert sc > sf + 10


def test_coarse_basis_rank_and_operator(tiny, floating):
    """The greedy basis keeps exactly rank(Z) columns (SVD) and gives the same
    coarse operator as the pseudo-inverse: Z_K E_K^-1 Z_K^T = Z E^+ Z^T."""
    for s, dec in (tiny, floating):
        pre = geneo.TwoLevel(dec, tau=10.0, nev_max=20)
        Z = pre.Z.toarray()
        sv = np.linalg.svd(Z, compute_uv=False)
        assert pre.rank == int((sv > 1e-10 * sv[0]).sum())
        Zk = Z[:, pre.kept]
        C1 = Zk @ np.linalg.solve(pre.E[np.ix_(pre.kept, pre.kept)], Zk.T)
        C2 = Z @ np.linalg.pinv(pre.E, rcond=1e-12, hermitian=True) @ Z.T
        assert np.allclose(C1, C2, atol=1e-7 * abs(C1).max())


def test_two_level_preconditioner_properties(tiny):
    """M_AS,2^-1 is symmetric positive definite, P_0 is a projection with
    P_0 Z = Z, and the spectrum of M^-1 A lies in [1/(1 + k1 tau), k0]
    (main theorem, Section 3.2, with c_R = k0 from the continuity lemma)."""
    s, dec = tiny
    tau = 10.0
    pre = geneo.TwoLevel(dec, tau=tau, nev_max=0)
    Minv = pre.matrix()
    assert np.allclose(Minv, Minv.T, atol=1e-10 * abs(Minv).max())
    A = s.A.toarray()
    Zk = pre.Z.toarray()[:, pre.kept]
    P0 = Zk @ np.linalg.solve(Zk.T @ A @ Zk, Zk.T @ A)
    assert np.allclose(P0 @ P0, P0, atol=1e-8)
    assert np.allclose(P0 @ Zk, Zk, atol=1e-8)
    ev = np.sort(sla.eigvals(Minv @ A).real)
    k0, k1 = geneo.k0_k1(dec)
    assert ev[0] >= 1.0 / (1.0 + k1 * tau) - 1e-10
    assert ev[-1] <= k0 + 1e-10
    assert np.linalg.eigvalsh(0.5 * (Minv + Minv.T)).min() > 0


def test_pcg_converges_to_direct_solution(floating):
    s, dec = floating
    pre = geneo.TwoLevel(dec, tau=10.0, nev_max=20)
    b = np.random.default_rng(7).standard_normal(s.n)
    x, it, hist = geneo.pcg(s.A, b, pre.apply, rtol=1e-8)
    xs = spla.spsolve(s.A.tocsc(), b)
    assert np.linalg.norm(b - s.A @ x) <= 1.5e-8 * np.linalg.norm(b)
    assert np.linalg.norm(x - xs) <= 1e-6 * np.linalg.norm(xs)
    # the two-level method needs fewer iterations than one-level AS
    _, it1, _ = geneo.pcg(s.A, b, geneo.TwoLevel(dec, variant="as").apply, rtol=1e-8)
    assert it < it1


@pytest.fixture(scope="module")
def stiff():
    # small gamma and high contrast: kappa(A_i) large enough that an FP32
    # factor leaves a visible error for the refinement to remove
    return _case((4, 4, 4), (2, 2, 1), gamma=1e-4, contrast=1e4, seed=3)[1]


def test_fp32_refinement_step(stiff):
    """One FP64 refinement step after an FP32 Cholesky solve: the error
    operator is squared, e1 = (I - Ahat^-1 A) e0, so in the A-norm
    ||e1||_A <= rho^2 ||x||_A with rho the spectral radius of I - Ahat^-1 A
    (Ahat^-1 A is A-self-adjoint); the map equals 2 Ahat^-1 - Ahat^-1 A Ahat^-1
    and is symmetric."""
    tl = geneo.TwoLevel(stiff, variant="as", local_precision="fp32_refine1")
    rng = np.random.default_rng(0)
    for i in range(stiff.N):
        A = tl.local_A[i]
        L = tl.local_L[i]
        assert L.dtype == np.float64 and np.array_equal(L.astype(np.float32).astype(np.float64), L)
        n = A.shape[0]
        x = rng.standard_normal(n)
        r = A @ x
        yhat = sla.cho_solve((L, True), r)
        y = tl.local_solve(i, r)
        anorm = lambda v: float(np.sqrt(v @ (A @ v)))
        rho = tl.fp32_rho(i)
        assert 0.0 < rho < 1.0
        e0, e1 = anorm(x - yhat), anorm(x - y)
        assert e0 <= rho * anorm(x) * (1 + 1e-6) + 1e-12 * anorm(x)
        assert e1 <= rho ** 2 * anorm(x) * (1 + 1e-6) + 1e-12 * anorm(x)
        assert e1 < e0
        Ahinv = sla.cho_solve((L, True), np.eye(n))
        Mref = 2 * Ahinv - Ahinv @ A @ Ahinv
        Mcol = np.column_stack([tl.local_solve(i, e) for e in np.eye(n)[:40]])
        assert np.abs(Mcol - Mref[:, :40]).max() <= 1e-9 * np.abs(Mref).max()
        assert np.abs(Mref - Mref.T).max() <= 1e-9 * np.abs(Mref).max()


def test_fp32_refined_two_level_pcg(stiff):
    """The FP32-refined preconditioner keeps PCG within one iteration of FP64."""
    s = stiff.sys
    b = np.random.default_rng(1).standard_normal(s.n)
    it = {}
    for prec in ("fp64", "fp32_refine1"):
        tl = geneo.TwoLevel(stiff, local_precision=prec)
        x, it[prec], _ = geneo.pcg(s.A, b, tl.apply, rtol=1e-8)
        assert np.linalg.norm(b - s.A @ x) <= 1.01e-8 * np.linalg.norm(b)
    assert it["fp32_refine1"] <= it["fp64"] + 1


def test_node_gradient_rayleigh_quotient_bounds_scaled_condition(tiny, floating):
    """The FP32 conditioning check's premise, on the oracle's matrices: for a
    free node whose edges all lie in Omega_i, v = G e_node is annihilated by
    the curl-curl part (K G = 0), so v^T A_i v = gamma v^T M v, and
    q = v^T A_i v / v^T diag(A_i) v bounds the smallest eigenvalue of
    D^-1/2 A_i D^-1/2 from above (a Rayleigh quotient); that matrix has a
    unit diagonal, so its largest eigenvalue is >= 1 and 1/q <= its
    condition number.  The bound is tight within a factor ~50 here."""
    for s, dec in (tiny, floating):
        A = s.A.tocsr()
        G = s.G.tocsc()
        for i in range(dec.N):
            d = np.asarray(dec.dofs[i])
            inside = np.zeros(s.n, bool)
            inside[d] = True
            Ai = A[d][:, d].toarray()
            dg = np.diag(Ai)
            r = 1.0 / np.sqrt(dg)
            ev = np.linalg.eigvalsh(Ai * r[:, None] * r[None, :])
            kappa = ev[-1] / ev[0]
            qmin = np.inf
            for c in np.unique(G[d].nonzero()[1]):
                rows = G[:, c].nonzero()[0]
                if not inside[rows].all():
                    continue
                v = G[:, c].toarray().ravel()
                assert abs(v @ (s.K @ v)) <= 1e-12 * (np.abs(v) @ (abs(s.K) @ np.abs(v)))
                assert np.isclose(v @ (A @ v), s.gamma * (v @ (s.M @ v)), rtol=1e-10)
                q = (v @ (A @ v)) / (v @ (A.diagonal() * v))
                assert q >= ev[0] * (1 - 1e-10)
                qmin = min(qmin, q)
            assert np.isfinite(qmin)
            assert 1.0 / qmin <= kappa * (1 + 1e-10)
            assert kappa <= 50.0 / qmin


def test_gmres_minimal_residual_and_special_cases():
    """Right-preconditioned GMRES (the paper's solver): on a non-symmetric
    system it reaches the direct solution within n steps, its residual
    history never increases (minimal residual over a growing Krylov space),
    the residual it reads from the rotations is the true ||b - A x||; the
    exact inverse as preconditioner solves in one step; restarted, it
    reaches the same solution."""
    rng = np.random.default_rng(3)
    n = 40
    A = 8.0 * np.eye(n) + rng.standard_normal((n, n))
    b = rng.standard_normal(n)
    xs = np.linalg.solve(A, b)
    x, it, hist = geneo.gmres(A, b, rtol=1e-12)
    assert it <= n
    assert all(hist[k + 1] <= hist[k] * (1 + 1e-12) for k in range(len(hist) - 1))
    true = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
    assert abs(true - hist[-1]) <= 1e-3 * hist[-1] + 1e-15
    assert np.linalg.norm(x - xs) <= 1e-10 * np.linalg.norm(xs)
    Ainv = np.linalg.inv(A)
    x1, it1, _ = geneo.gmres(A, b, M=lambda v: Ainv @ v, rtol=1e-10)
    assert it1 == 1 and np.linalg.norm(x1 - xs) <= 1e-10 * np.linalg.norm(xs)
    x2, it2, _ = geneo.gmres(A, b, rtol=1e-12, restart=7, maxit=2000)
    assert it2 > it and np.linalg.norm(x2 - xs) <= 1e-10 * np.linalg.norm(xs)


def test_restricted_weights(tiny):
    """weight="pou" puts D_i into the one-level sum: the operator is no longer
    symmetric (with identity weights it is); with a single subdomain
    (D = I, A_1 = A) it is A^-1 itself and GMRES stops after one step;
    as right preconditioner of the two-level method it reaches the direct
    solution on the tiny case."""
    s, dec = tiny
    n = s.n
    E = np.eye(n)
    sym = geneo.TwoLevel(dec, variant="as")
    ras = geneo.TwoLevel(dec, variant="as", weight="pou")
    Ms = np.column_stack([sym.one_level(e) for e in E])
    Mr = np.column_stack([ras.one_level(e) for e in E])
    assert np.abs(Ms - Ms.T).max() <= 1e-10 * np.abs(Ms).max()
    assert np.abs(Mr - Mr.T).max() >= 1e-3 * np.abs(Mr).max()
    s1, dec1 = _case((4, 4, 4), (1, 1, 1))
    one = geneo.TwoLevel(dec1, variant="as", weight="pou")
    b = np.random.default_rng(4).standard_normal(s1.n)
    xs = spla.splu(s1.A.tocsc()).solve(b)
    assert np.linalg.norm(one.one_level(b) - xs) <= 1e-10 * np.linalg.norm(xs)
    x, it, _ = geneo.gmres(s1.A, b, M=one.apply, rtol=1e-10)
    assert it == 1 and np.linalg.norm(x - xs) <= 1e-9 * np.linalg.norm(xs)
    two = geneo.TwoLevel(dec, weight="pou")
    b = np.random.default_rng(5).standard_normal(n)
    xs = spla.splu(s.A.tocsc()).solve(b)
    x, it, hist = geneo.gmres(s.A, b, M=two.apply, rtol=1e-10)
    assert hist[-1] <= 1e-10 and it < n
    assert np.linalg.norm(x - xs) <= 1e-7 * np.linalg.norm(xs)


def test_mixed_beam_geneo_columns_are_the_relative_harmonic_field():
    """The paper's beam with Neumann conditions on the lateral faces -y/+y
    (Section 4, Numerical results; here N = 4 strips at h = 1/8): an
    interior strip's Dirichlet boundary (faces z = 0 and z = 1) has two
    components, so grad z is curl-free, satisfies the strip's boundary
    conditions and is no gradient of a free nodal function (z is 1 on the
    Dirichlet face z = 1).  Its B-orthogonal part off span(G_i), h, has
    B h = gamma M h but D_i breaks its curl-freeness under Atilde: the
    filtered GEVP (eq. (eigAtildeBAS)) has exactly one eigenvalue above tau
    there, of order 1 / gamma, whose eigenvector is h (B-cosine 1 - 1e-5).
    The end strips (Dirichlet face x = 0 or x = L: grad z is not admissible)
    and every strip of the all-Dirichlet beam select nothing.  This is the
    N - 2 GenEO columns of the mixed beam."""
    for bc, expect in (("mixed", [0, 1, 1, 0]), ("all", [0, 0, 0, 0])):
        w = W.paper_beam(4, bc=bc, cells=8)
        s = fem.System(w.mesh, w.mu, w.eps, w.gamma, w.dirichlet)
        dec = decomp.Decomposition(s, decomp.partition_cells(w), w.overlap)
        assert dec.N == 4
        for i in range(4):
            Gi, _, _ = dec.G_local(i)
            A, B, D = dec.A_dir(i).toarray(), dec.A_neu(i).toarray(), dec.D[i]
            lam, V, sel = geneo.gevp(A, B, D, Gi, w.tau, w.nev_max)
            assert sel == expect[i], (bc, i, sel, lam[:3])
            if sel:
                assert lam[0] > 0.1 / w.gamma and lam[1] < w.tau
                ab = s.edges[s.free_edges[dec.dofs[i]]]
                z = s.mesh["xyz"][:, 2]
                t = z[ab[:, 1]] - z[ab[:, 0]]          # edge dofs of grad z
                Gd = Gi.toarray()
                h = t - Gd @ np.linalg.solve(Gd.T @ B @ Gd, Gd.T @ (B @ t))
                v = V[:, 0]
                cos = abs(v @ B @ h) / np.sqrt((v @ B @ v) * (h @ B @ h))
                assert cos > 1 - 1e-4, cos


@pytest.mark.parametrize("cfg", ["small_channels", "small_floating", "small_hole"])
def test_deflated_pcg_follows_the_balanced_iterates(cfg):
    """PCG with the deflated form (I - Q A) M_AS^-1 + Q from x0 = Q b against
    PCG with M_AS,2 (eq. (AS2)) from x0 = 0: the same iteration count, the
    same solution to 1e-7 relative, and Z^T r stays at rounding level along
    the deflated run (the property that makes the two operators agree)."""
    w = W.make(cfg)
    s = fem.System(w.mesh, w.mu, w.eps, w.gamma, w.dirichlet)
    dec = decomp.Decomposition(s, decomp.partition_cells(w), w.overlap)
    opc = geneo.TwoLevel(dec, tau=w.tau, nev_max=w.nev_max)
    b = w.rhs(s.n)
    xb, itb, _ = geneo.pcg(s.A, b, opc.apply, rtol=1e-8)
    zr = []
    zn = spla.norm(opc.Z)   # Frobenius norm, >= the spectral one

    def M(r):
        zr.append(np.linalg.norm(opc.Z.T @ r) / (zn * np.linalg.norm(r)))
        return opc.apply_deflated(r)

    xd, itd, _ = geneo.pcg(s.A, b, M, rtol=1e-8, x0=opc.deflated_start(b))
    assert itd == itb, (itd, itb)
    assert np.linalg.norm(xd - xb) <= 1e-7 * np.linalg.norm(xb)
    assert max(zr) <= 1e-10
