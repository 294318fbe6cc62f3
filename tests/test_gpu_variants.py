"""GPU parity of the paper's comparison variants (Section 4, Numerical
results) against the oracle, on the same kernels as the method: the global
near-kernel coarse spaces (Z = G, alone and with the GenEO vectors), the
classical GenEO pencil (eq. (eigGenEOClassis)), the restricted one-level
term with the partition of unity (eq. (RAS)) and right-preconditioned GMRES
(the paper's Krylov method), with and without restarts."""
import numpy as np
import pytest

import workloads as W
from cases import lib_problem, oracle_problem, rel, solve_tol, to_dev

pytestmark = pytest.mark.gpu

CASES = ["small_channels", "small_hole"]


@pytest.fixture(scope="module")
def g():
    import torch
    from paper_2311_18783_amd import geneo
    assert torch.cuda.is_available()
    ctx = geneo.Context(0)
    yield geneo, ctx
    ctx.close()


def _apply(ctx, pc, r):
    import torch
    z = torch.zeros(r.size, dtype=torch.float64, device="cuda:0")
    ctx.apply(pc, to_dev(r), z)
    torch.cuda.synchronize()
    return z.cpu().numpy()


@pytest.mark.parametrize("cfg", CASES)
@pytest.mark.parametrize("variant", ["nk", "nk_geneo"])
def test_global_near_kernel_coarse_space(g, cfg, variant):
    """Z = G (every free node's gradient), with or without the GenEO
    vectors: coarse size and rank equal the oracle's, the apply matches
    (1e-10 without eigenvectors, 1e-4 with), PCG needs as many iterations."""
    import torch
    from oracle import geneo as og
    geneo, ctx = g
    w = W.make(cfg)
    print("variant", variant, cfg, flush=True)
    s, odec = oracle_problem(w)
    opc = og.TwoLevel(odec, tau=w.tau, nev_max=w.nev_max, variant=variant)
    sysm, dec = lib_problem(ctx, w)
    kind = geneo.COARSE_NK if variant == "nk" else geneo.COARSE_NK_GENEO
    pc = ctx.setup(sysm, dec, tau=w.tau, nev_max=w.nev_max, coarse=kind)
    info = pc.info()
    assert info.n0 == opc.n0 and info.n0_rank == opc.rank, (info.n0, opc.n0, info.n0_rank, opc.rank)
    assert info.n_geneo == opc.n_geneo
    r = np.random.default_rng(21).standard_normal(s.n)
    e = rel(_apply(ctx, pc, r), opc.apply(r))
    # without eigenvectors the two applies differ by the local solves' rounding (10 eps max kappa(A_i))
    tol = solve_tol(odec) if variant == "nk" else 1e-4
    print("apply rel err", e, "tol", tol, flush=True)
    assert e <= tol
    b = w.rhs(s.n)
    x = torch.zeros(s.n, dtype=torch.float64, device="cuda:0")
    si = ctx.solve(sysm, pc, to_dev(b), x, rtol=1e-8)
    xo, ito, _ = og.pcg(s.A, b, opc.apply, rtol=1e-8)
    print("iterations", si.iterations, "oracle", ito, flush=True)
    assert si.iterations == ito
    assert rel(x.cpu().numpy(), xo) <= 1e-7


@pytest.mark.parametrize("cfg", ["small_channels", "small_mixed"])
def test_classical_pencil_eigenvalues(g, cfg):
    """The classical pencil D_j A_j D_j V = lambda A_j^Neu V: eigenvalues above
    tau (at most 12; its spectrum above tau is wide, so the eigensolver block
    carries 12 guard vectors) agree with the oracle's dense eigensolver to 1e-8,
    the selected counts agree outside a tie band of 1e-6 around tau, and the
    coarse space is at least as large as the filtered pencil's (the
    near-kernel is not projected out)."""
    from oracle import geneo as og
    geneo, ctx = g
    w = W.make(cfg)
    print("classical", cfg, flush=True)
    s, odec = oracle_problem(w)
    sysm, dec = lib_problem(ctx, w)
    nev = 12
    pcc = ctx.setup(sysm, dec, tau=w.tau, nev_max=nev, lobpcg_guard=12, classical=1)
    pcf = ctx.setup(sysm, dec, tau=w.tau, nev_max=nev, lobpcg_guard=12)
    assert pcc.info().lobpcg_unconverged == 0
    for i in range(odec.N):
        Gi, _, _ = odec.G_local(i)
        lam_o, _, sel_o = og.gevp(odec.A_dir(i).toarray(), odec.A_neu(i).toarray(), odec.D[i], Gi, w.tau,
                                  nev, classical=True)
        lam_g, sel_g = pcc.eigs(i)
        near = np.abs(lam_o[:nev + 1] / w.tau - 1.0) < 1e-6
        if not near.any():
            assert sel_g == sel_o, (i, sel_g, sel_o)
        m = min(sel_g, sel_o)
        if m:
            err = np.abs(lam_g[:m] - lam_o[:m]) / np.abs(lam_o[:m])
            assert err.max() <= 1e-8, (i, err.max())
    assert pcc.info().n_geneo >= pcf.info().n_geneo
    print("GenEO columns classical", pcc.info().n_geneo, "filtered", pcf.info().n_geneo, flush=True)


@pytest.mark.parametrize("cfg", CASES)
@pytest.mark.parametrize("weight,restart", [("pou", 0), ("identity", 0), ("pou", 8)])
def test_gmres_matches_oracle(g, cfg, weight, restart):
    """Right-preconditioned GMRES at rtol 1e-6 (the paper's solver) with the
    restricted (eq. (RAS)) or the plain one-level term in the two-level
    preconditioner, without and with restarts: the GPU apply matches the
    oracle's (1e-4, eigenvector accuracy), GMRES needs as many iterations as
    the oracle's GMRES, and the true residual meets the tolerance."""
    import torch
    from oracle import geneo as og
    geneo, ctx = g
    w = W.make(cfg)
    print("gmres", cfg, weight, restart, flush=True)
    s, odec = oracle_problem(w)
    opc = og.TwoLevel(odec, tau=w.tau, nev_max=w.nev_max, weight=weight)
    sysm, dec = lib_problem(ctx, w)
    pc = ctx.setup(sysm, dec, tau=w.tau, nev_max=w.nev_max,
                   one_level_weight=geneo.WEIGHT_POU if weight == "pou" else geneo.WEIGHT_IDENTITY)
    r = np.random.default_rng(23).standard_normal(s.n)
    assert rel(_apply(ctx, pc, r), opc.apply(r)) <= 1e-4
    b = w.rhs(s.n)
    x = torch.zeros(s.n, dtype=torch.float64, device="cuda:0")
    si = ctx.solve(sysm, pc, to_dev(b), x, rtol=1e-6, method=geneo.GMRES, restart=restart)
    xo, ito, _ = og.gmres(s.A, b, opc.apply, rtol=1e-6, restart=restart or None)
    xg = x.cpu().numpy()
    tr = np.linalg.norm(b - s.A @ xg) / np.linalg.norm(b)
    print("gmres iterations", si.iterations, "oracle", ito, "true residual", tr, "x vs oracle", rel(xg, xo),
          flush=True)
    assert si.iterations == ito
    assert tr <= 1.01e-6


def test_level_schedule_matches_step_schedule_on_strips(g):
    """Sixteen strips of the paper's beam (h = 1/16) in nested-dissection
    order: the coarse factor run by elimination-tree levels (forced) and by
    panel steps keeps the same columns, and the two preconditioners agree on
    a random vector to 1e-9 and need the same PCG iterations."""
    import torch
    geneo, ctx = g
    w = W.make("beam16")
    print("level schedule", w.name, flush=True)
    sysm, dec = lib_problem(ctx, w)
    pl = ctx.setup(sysm, dec, tau=w.tau, nev_max=w.nev_max, coarse_order=geneo.ORDER_NESTED_DISSECTION,
                   coarse_schedule=geneo.SCHEDULE_LEVELS)
    ps = ctx.setup(sysm, dec, tau=w.tau, nev_max=w.nev_max, coarse_order=geneo.ORDER_NESTED_DISSECTION,
                   coarse_schedule=geneo.SCHEDULE_STEPS)
    il, is_ = pl.info(), ps.info()
    print("levels", il.coarse_levels, "schedules", il.coarse_schedule_used, is_.coarse_schedule_used, "rank",
          il.n0_rank, is_.n0_rank, "nd levels", il.coarse_nd_levels, flush=True)
    assert il.coarse_schedule_used == geneo.SCHEDULE_LEVELS and is_.coarse_schedule_used == geneo.SCHEDULE_STEPS
    assert il.coarse_nd_levels >= 2 and il.coarse_levels > 1
    assert il.n0_rank == is_.n0_rank
    n = sysm.info().n
    r = np.random.default_rng(37).standard_normal(n)
    d = rel(_apply(ctx, pl, r), _apply(ctx, ps, r))
    print("apply difference", d, flush=True)
    assert d <= 1e-9
    b = w.rhs(n)
    its = []
    for pc in (pl, ps):
        x = torch.zeros(n, dtype=torch.float64, device="cuda:0")
        its.append(ctx.solve(sysm, pc, to_dev(b), x, rtol=1e-8).iterations)
    assert its[0] == its[1], its


def test_nested_dissection_order_keeps_the_coarse_space(g):
    """The nested-dissection elimination order of the coarse columns on a
    chain of six strip subdomains (12 x 4 x 4 beam, Neumann lateral faces):
    the dissection has a level, the coarse space and its rank are unchanged
    (a clear gap in the Schur pivots), the apply still matches the oracle's,
    PCG needs the oracle's iteration count, and the dependency chain of the
    coarse triangular solves is no longer than in the natural order (on
    this small chain every group fits one or two 128-column tiles)."""
    import torch
    from oracle import geneo as og
    geneo, ctx = g
    w = W.make("small_mixed", partition={"kind": "box", "p": (6, 1, 1)})
    print("nd order", w.name, flush=True)
    s, odec = oracle_problem(w)
    opc = og.TwoLevel(odec, tau=w.tau, nev_max=w.nev_max)
    sysm, dec = lib_problem(ctx, w)
    pn = ctx.setup(sysm, dec, tau=w.tau, nev_max=w.nev_max, coarse_order=geneo.ORDER_NATURAL)
    pd = ctx.setup(sysm, dec, tau=w.tau, nev_max=w.nev_max, coarse_order=geneo.ORDER_NESTED_DISSECTION)
    inn, ind = pn.info(), pd.info()
    print("levels", ind.coarse_nd_levels, "solve depth natural", inn.coarse_solve_depth, "nd", ind.coarse_solve_depth,
          flush=True)
    assert ind.coarse_nd_levels >= 1 and inn.coarse_nd_levels == 0
    assert ind.n0 == opc.n0 and ind.n0_rank == opc.rank == inn.n0_rank
    assert ind.coarse_solve_depth <= inn.coarse_solve_depth
    r = np.random.default_rng(29).standard_normal(s.n)
    assert rel(_apply(ctx, pd, r), opc.apply(r)) <= 1e-4
    assert rel(_apply(ctx, pd, r), _apply(ctx, pn, r)) <= 1e-8
    b = w.rhs(s.n)
    x = torch.zeros(s.n, dtype=torch.float64, device="cuda:0")
    si = ctx.solve(sysm, pd, to_dev(b), x, rtol=1e-8)
    _, ito, _ = og.pcg(s.A, b, opc.apply, rtol=1e-8)
    assert si.iterations == ito
