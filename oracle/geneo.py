"""Oracle: local projections, the filtered GenEO eigenproblem, the coarse
space, the two-level additive Schwarz preconditioner and PCG.

Paper passages:
  * b_i(U,V) = (A_i U, V) and xi_0i, the b_i-orthogonal projection onto
    span(G_i) (Section 2, eq. (b), Definition of orthogonal projections and
    complements, eq. (Giortho), and the lemma with eq. (inverseBw));
  * the generalised eigenproblem (I - xi_j^T) D_j A_j D_j (I - xi_j) V =
    lambda A_j^Neu V, eigenvectors with lambda > tau, coarse vectors
    R_j^T D_j (I - xi_j) V (Section 3.2, GEVP "tauthresholdAS",
    eq. (eigAtildeBAS)); tau = 10 (Section 4, Numerical results);
  * the classical GenEO pencil D_j A_j D_j V = lambda A_j^Neu V (Section 3.2,
    eq. (eigGenEOClassis)) for comparison;
  * the split near-kernel space V_G = span(R_i^T D_i G_i) (Definition
    "Split near-kernel coarse space") and V_0 = V_G + V_GenEO (eq. (V0GenEOAS));
  * E = Z^T A Z, P_0 = Z E^-1 Z^T A and the balanced two-level form
    M^-1 = Z E^-1 Z^T + (I - P_0) sum_i R_i^T A_i^-1 R_i (I - P_0^T)
    (Section 2, eq. (AS) and eq. (AS2); Section 3.2, the explicit M_AS,2);
  * the condition number bound kappa <= (1 + k1 tau) k0 (Section 3.2, main
    theorem; k0 eq. (k0), k1 after it).

The paper leaves the local solver open (Section 2 only needs A_i^-1); the
"fp32_refine1" local precision is the mixed-precision variant of the
measured workload: A_i factored in FP32, then one FP64 refinement step
y = yhat + Ahat^-1 (r_i - A_i yhat), yhat = Ahat^-1 r_i, which as a map is
2 Ahat^-1 - Ahat^-1 A_i Ahat^-1 (symmetric; positive definite exactly when
rho(I - Ahat^-1 A_i) < 1).  The triangular solves use the FP32 factor with
FP64 vectors.

Readings: the paper solves with right-preconditioned GMRES at rtol 1e-6
(Section 4, Numerical results, with the reason that the residual is then minimised in the same
norm whatever the preconditioner); `gmres` below is that solver.  The
measured path runs preconditioned conjugate gradients (the preconditioner
is symmetric positive definite) from x0 = 0, stopping at the first iterate
with ||r_k||_2 <= rtol ||b||_2 (recurrence residual); `apply_deflated` with
x0 = Q b (`deflated_start`) is the one-coarse-solve form with the same PCG
iterates in exact arithmetic (every residual then has Z^T r = 0, where it
equals M_AS,2).  weight="pou" puts the
partition of unity D_i of Section 2 into the one-level sum,
sum_i R_i^T D_i A_i^-1 R_i (the restricted additive Schwarz variant; not
symmetric, so it goes with GMRES).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def xi_projection(Ai, Gi):
    """xi_0i = G_i (G_i^T A_i G_i)^-1 G_i^T A_i, dense n_i x n_i: the
    A_i-orthogonal projection onto span(G_i) (Section 2)."""
    Ai = np.asarray(Ai)
    Gd = Gi.toarray() if sp.issparse(Gi) else np.asarray(Gi)
    S = Gd.T @ Ai @ Gd
    return Gd @ np.linalg.solve(S, Gd.T @ Ai)


def filtered_pencil(Ai, Neu, Di, Gi):
    """Left and right matrices of the filtered GEVP (eq. (eigAtildeBAS))."""
    Ai = np.asarray(Ai)
    xi = xi_projection(Ai, Gi)
    Q = np.eye(Ai.shape[0]) - xi
    DAD = Di[:, None] * Ai * Di[None, :]
    At = Q.T @ DAD @ Q
    At = 0.5 * (At + At.T)
    return At, np.asarray(Neu)


def gevp(Ai, Neu, Di, Gi, tau=10.0, nev_max=20, classical=False):
    """Solve the local GEVP with a dense symmetric-definite eigensolver.

    Returns (lam_desc, V_desc, sel): all eigenvalues in decreasing order with
    B-normalised eigenvectors, and the number selected: those with
    lambda > tau, at most nev_max (0 = no cap)."""
    if classical:
        Ai = np.asarray(Ai)
        At = Di[:, None] * Ai * Di[None, :]
        B = np.asarray(Neu)
    else:
        At, B = filtered_pencil(Ai, Neu, Di, Gi)
    lam, V = sla.eigh(At, B)
    lam, V = lam[::-1], V[:, ::-1]
    sel = int((lam > tau).sum())
    if nev_max:
        sel = min(sel, nev_max)
    return lam, V, sel


def geneo_vectors(Ai, Gi, Di, V):
    """Local coarse vectors D_i (I - xi_i) V (to be extended by R_i^T)."""
    xi = xi_projection(np.asarray(Ai), Gi)
    return Di[:, None] * (V - xi @ V)


def greedy_cholesky(E, drop_tol=1e-7):
    """Cholesky factor of E restricted to a basis chosen greedily from the
    columns of Z, left to right.

    The columns R_i^T D_i G_i span V_G but are not linearly independent in
    general (several subdomains hold the same node where the partition of
    unity is locally proportional, or D_i vanishes on a node's whole edge
    star), so E = Z^T A Z is only semi-definite.  Column j is kept iff its
    squared A-distance to the span of the kept columns before it (the Schur
    complement pivot) exceeds drop_tol * E_jj; the kept columns are then a
    basis of V_0 and Z_K E_KK^-1 Z_K^T is the coarse operator of V_0
    (identical to Z E^+ Z^T).  Returns (L of E_KK, boolean mask of kept)."""
    S = np.array(E, dtype=np.float64, copy=True)
    n = S.shape[0]
    d = np.diag(S).copy()
    kept = np.zeros(n, dtype=bool)
    for j in range(n):
        p = S[j, j]
        if not (p > drop_tol * d[j]) or d[j] <= 0:
            S[j:, j] = 0.0
            S[j, j:] = 0.0
            continue
        kept[j] = True
        col = S[j + 1:, j] / np.sqrt(p)
        S[j + 1:, j + 1:] -= np.outer(col, col)
    Ek = E[np.ix_(kept, kept)]
    return sla.cholesky(Ek, lower=True), kept


class TwoLevel:
    """M_AS,2 with the SNK (+ GenEO) coarse space, built from a Decomposition.

    variant: 'snk_geneo' (the method), 'snk' (tau = infinity), 'as' (one
    level, no coarse space), 'nk' / 'nk_geneo' (Z from the global G)."""

    def __init__(self, dec, tau=10.0, nev_max=20, variant="snk_geneo", classical=False,
                 drop_tol=1e-7, local_precision="fp64", weight="identity"):
        self.dec = dec
        if weight not in ("identity", "pou"):
            raise ValueError(weight)
        self.weight = weight
        sysm = dec.sys
        n = sysm.n
        self.variant = variant
        if local_precision not in ("fp64", "fp32_refine1"):
            raise ValueError(local_precision)
        self.local_precision = local_precision
        self.local_L = []
        self.local_A = []
        self.eig = []
        self.G_locals = []
        cols_snk = []
        geneo_cols = []
        self.geneo_counts = []
        for i in range(dec.N):
            Ai = dec.A_dir(i).toarray()
            if local_precision == "fp32_refine1":
                self.local_L.append(sla.cholesky(Ai.astype(np.float32), lower=True).astype(np.float64))
                self.local_A.append(Ai)
            else:
                self.local_L.append(sla.cholesky(Ai, lower=True))
            Gi, gnodes, _ = dec.G_local(i)
            self.G_locals.append((Gi, gnodes))
            if variant in ("snk", "snk_geneo"):
                Zi = sp.diags(dec.D[i]) @ Gi            # D_i G_i, n_i x p_i
                cols_snk.append((dec.dofs[i], Zi.tocoo()))
            if variant in ("snk_geneo", "nk_geneo"):
                Neu = dec.A_neu(i).toarray()
                lam, V, sel = gevp(Ai, Neu, dec.D[i], Gi, tau, nev_max, classical=classical)
                self.eig.append((lam, V, sel))
                self.geneo_counts.append(sel)
                if sel:
                    W = geneo_vectors(Ai, Gi, dec.D[i], V[:, :sel])
                    full = np.zeros((n, sel))
                    full[dec.dofs[i]] = W
                    geneo_cols.append(full)
        blocks = []
        if variant in ("snk", "snk_geneo"):
            r, c, v = [], [], []
            off = 0
            for dofs, Zi in cols_snk:
                r.append(dofs[Zi.row])
                c.append(Zi.col + off)
                v.append(Zi.data)
                off += Zi.shape[1]
            blocks.append(sp.csc_matrix((np.concatenate(v), (np.concatenate(r), np.concatenate(c))),
                                        shape=(n, off)))
        elif variant in ("nk", "nk_geneo"):
            blocks.append(sysm.G.tocsc())
        self.n_snk = blocks[0].shape[1] if blocks else 0
        if geneo_cols:
            blocks.append(sp.csc_matrix(np.concatenate(geneo_cols, axis=1)))
        self.n_geneo = sum(g.shape[1] for g in geneo_cols)
        if blocks:
            self.Z = sp.hstack(blocks).tocsc()
            self.AZ = (sysm.A @ self.Z).tocsc()
            E = (self.Z.T @ self.AZ).toarray()
            self.E = 0.5 * (E + E.T)
            self.n0 = E.shape[0]
            self.E_L, self.kept = greedy_cholesky(self.E, drop_tol)
            self.rank = int(self.kept.sum())
        else:
            self.Z = None
            self.n0 = 0

    def coarse_solve(self, v):
        """E^+ v restricted to the kept (basis) columns; dropped entries 0."""
        k = self.kept
        out = np.zeros_like(v)
        out[k] = sla.cho_solve((self.E_L, True), v[k])
        return out

    def local_solve(self, i, ri):
        """A_i^-1 r_i: FP64 Cholesky, or FP32 Cholesky plus one FP64 refinement step."""
        L = self.local_L[i]
        y = sla.cho_solve((L, True), ri)
        if self.local_precision == "fp32_refine1":
            y = y + sla.cho_solve((L, True), ri - self.local_A[i] @ y)
        return y

    def one_level(self, r):
        """sum_i R_i^T A_i^-1 R_i r (eq. (AS)), dense Cholesky solves; with
        weight="pou", sum_i R_i^T D_i A_i^-1 R_i r (restricted variant)."""
        y = np.zeros_like(r)
        for i in range(len(self.local_L)):
            d = self.dec.dofs[i]
            yi = self.local_solve(i, r[d])
            Di = self.dec.D[i] if yi.ndim == 1 else self.dec.D[i][:, None]
            y[d] += Di * yi if self.weight == "pou" else yi
        return y

    def fp32_rho(self, i):
        """rho(I - Ahat_i^-1 A_i) of the FP32 factor (dense eigenvalues; small cases)."""
        L = self.local_L[i]
        T = np.eye(L.shape[0]) - sla.cho_solve((L, True), self.local_A[i])
        return float(np.abs(np.linalg.eigvals(T)).max())

    def apply(self, r):
        """z = M_AS,2^-1 r = Z E^-1 Z^T r + (I - P_0) M_AS^-1 (I - P_0^T) r."""
        if self.Z is None:
            return self.one_level(r)
        c = self.coarse_solve(self.Z.T @ r)
        y = self.one_level(r - self.AZ @ c)
        c2 = self.coarse_solve(self.AZ.T @ y)
        return self.Z @ c + y - self.Z @ c2

    def apply_deflated(self, r):
        """z = M_AS^-1 r + Q (r - A M_AS^-1 r), Q = Z E^-1 Z^T: the deflated
        form (I - Q A) M_AS^-1 + Q of the preconditioner, one coarse solve.
        Where Z^T r = 0, (I - A Q) r = r and Q r = 0, and this equals
        M_AS,2^-1 r (eq. (AS2), as in `apply`); PCG from x0 = Q b keeps Z^T r = 0
        on every residual in exact arithmetic."""
        if self.Z is None:
            return self.one_level(r)
        y = self.one_level(r)
        t = r - self.dec.sys.A @ y
        return y + self.Z @ self.coarse_solve(self.Z.T @ t)

    def deflated_start(self, b):
        """x0 = Q b = Z E^-1 Z^T b (0 without a coarse space)."""
        if self.Z is None:
            return np.zeros_like(b)
        return self.Z @ self.coarse_solve(self.Z.T @ b)

    def matrix(self, block=512):
        """Dense M^-1, applied to blocks of unit vectors (small cases only)."""
        n = self.dec.sys.n
        out = np.empty((n, n))
        for j in range(0, n, block):
            e = np.zeros((n, min(block, n - j)))
            e[np.arange(j, j + e.shape[1]), np.arange(e.shape[1])] = 1.0
            out[:, j:j + e.shape[1]] = self.apply(e)
        return out


def pcg(A, b, M=None, rtol=1e-8, maxit=1000, x0=None):
    """Preconditioned conjugate gradients (Hestenes-Stiefel) from x0 (default
    0).  Stops at ||r_k|| <= rtol ||b||.  Returns (x, iterations, residual
    history ||r_k||/||b||)."""
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    r = b - A @ x if x0 is not None else b.copy()
    nb = np.linalg.norm(b)
    z = M(r) if M is not None else r.copy()
    p = z.copy()
    rz = r @ z
    hist = [1.0]
    for k in range(1, maxit + 1):
        q = A @ p
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        rn = np.linalg.norm(r)
        hist.append(rn / nb)
        if rn <= rtol * nb:
            return x, k, hist
        z = M(r) if M is not None else r.copy()
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, maxit, hist


def gmres(A, b, M=None, rtol=1e-6, maxit=1000, restart=None):
    """Right-preconditioned GMRES from x0 = 0 (the paper's solver, Section 4, Numerical results):
    Arnoldi with modified Gram-Schmidt on A M^-1, Givens rotations on the
    Hessenberg matrix, x = M^-1 V y.  With right preconditioning the
    minimised quantity is the true residual ||b - A x||_2, so the stop test
    ||b - A x_k|| <= rtol ||b|| reads the rotated right-hand side.  Restarts
    every `restart` steps (None: never).  Returns (x, iterations, residual
    history ||r_k||/||b||)."""
    n = b.shape[0]
    Mf = M if M is not None else (lambda v: v.copy())
    x = np.zeros_like(b)
    nb = np.linalg.norm(b)
    hist = [1.0]
    if nb == 0.0:
        return x, 0, hist
    m = restart or maxit
    it = 0
    while it < maxit:
        r = b - A @ x
        beta = np.linalg.norm(r)
        V = np.zeros((n, m + 1))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[:, 0] = r / beta
        k_done = 0
        for k in range(m):
            it += 1
            w = A @ Mf(V[:, k])
            for j in range(k + 1):
                H[j, k] = w @ V[:, j]
                w = w - H[j, k] * V[:, j]
            H[k + 1, k] = np.linalg.norm(w)
            if H[k + 1, k] > 0.0:
                V[:, k + 1] = w / H[k + 1, k]
            for j in range(k):
                t = cs[j] * H[j, k] + sn[j] * H[j + 1, k]
                H[j + 1, k] = -sn[j] * H[j, k] + cs[j] * H[j + 1, k]
                H[j, k] = t
            den = np.hypot(H[k, k], H[k + 1, k])
            cs[k] = H[k, k] / den
            sn[k] = H[k + 1, k] / den
            H[k, k] = den
            H[k + 1, k] = 0.0
            g[k + 1] = -sn[k] * g[k]
            g[k] = cs[k] * g[k]
            hist.append(abs(g[k + 1]) / nb)
            k_done = k + 1
            if abs(g[k + 1]) <= rtol * nb or it >= maxit:
                break
        y = sla.solve_triangular(H[:k_done, :k_done], g[:k_done])
        x = x + Mf(V[:, :k_done] @ y)
        if hist[-1] <= rtol:
            break
    return x, it, hist


def k0_k1(dec):
    """k0 = max_i #{j : R_j A R_i^T != 0} (eq. (k0)); k1 = the largest number
    of subdomains whose intersection has non-zero measure (cells shared)."""
    A = dec.sys.A
    N = dec.N
    k0 = 0
    for i in range(N):
        touched = np.zeros(dec.sys.n, bool)
        touched[A[dec.dofs[i]].indices] = True
        k0 = max(k0, sum(1 for j in range(N) if touched[dec.dofs[j]].any()))
    H = int(dec.sys.mesh["hex_of_tet"].max()) + 1
    cnt = np.zeros(H, np.int64)
    for c in dec.cells:
        cnt[c] += 1
    return k0, int(cnt.max())
