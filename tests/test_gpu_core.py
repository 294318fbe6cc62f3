"""GPU parity of the HIP library against the oracle: batched Cholesky,
assembly, decomposition, one- and two-level apply, PCG (SNK coarse space)."""
import numpy as np
import pytest

import workloads as W
from cases import lib_problem, oracle_problem, rel, solve_tol, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def g():
    import torch
    from paper_2311_18783_amd import geneo
    assert torch.cuda.is_available()
    ctx = geneo.Context(0)
    yield geneo, ctx
    ctx.close()


def _spd(n, rng, cond=1e4):
    Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
    ev = np.geomspace(1.0, cond, n)
    return (Q * ev) @ Q.T


def _pack(mats, dtype):
    sizes = [m.shape[0] for m in mats]
    lds = [((n + 127) // 128) * 128 for n in sizes]
    offs = np.cumsum([0] + [l * l for l in lds])
    buf = np.zeros(offs[-1], dtype=dtype)
    for m, ld, o in zip(mats, lds, offs):
        n = m.shape[0]
        full = np.eye(ld)
        full[:n, :n] = m
        buf[o:o + ld * ld] = full.T.ravel()       # column-major
    return buf, sizes, lds, offs[:-1]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_potrf_batched_ragged(g, prec):
    import torch
    geneo, ctx = g
    rng = np.random.default_rng(0)
    sizes = [1, 5, 127, 128, 129, 300, 700, 260]
    mats = [_spd(n, rng, 1e3 if prec == "fp32" else 1e6) for n in sizes]
    dt = np.float64 if prec == "fp64" else np.float32
    buf, sizes, lds, offs = _pack(mats, dt)
    print("potrf", prec, sizes, flush=True)
    A = torch.as_tensor(buf, device="cuda:0")
    ctx.potrf_batched(A, sizes, offs, geneo.FP64 if prec == "fp64" else geneo.FP32_REFINE1)
    torch.cuda.synchronize()
    out = A.cpu().numpy()
    for m, n, ld, o in zip(mats, sizes, lds, offs):
        L = np.tril(out[o:o + ld * ld].reshape(ld, ld).T)
        Lref = np.linalg.cholesky(m)
        tol = 1e-11 if prec == "fp64" else 2e-4
        assert np.abs(L[:n, :n] - Lref).max() <= tol * np.abs(Lref).max() * max(1, np.sqrt(n) / 4), (n, prec)
        if ld > n:
            assert np.allclose(L[n:, n:], np.eye(ld - n)) and np.abs(L[n:, :n]).max() == 0


def test_potrf_reports_non_spd(g):
    import torch
    geneo, ctx = g
    rng = np.random.default_rng(1)
    a = _spd(200, rng, 10.0)
    b = a.copy()
    b[150, 150] = -5.0
    buf, sizes, lds, offs = _pack([a, b], np.float64)
    A = torch.as_tensor(buf, device="cuda:0")
    with pytest.raises(geneo.GeneoError) as ei:
        ctx.potrf_batched(A, sizes, offs, geneo.FP64)
    assert ei.value.status == "ENOTSPD" and "matrix 1" in str(ei.value)


CASES = [1, "small_hole", "small_mixed", "small_floating"]


@pytest.mark.parametrize("cfg", CASES)
def test_assembly_and_partition_match_oracle(g, cfg):
    geneo, ctx = g
    w = W.make(cfg)
    print("assemble", cfg, flush=True)
    sysm, dec = lib_problem(ctx, w)
    s, odec = oracle_problem(w)
    A, fe = sysm.export()
    assert np.array_equal(fe, s.free_edges)
    assert np.array_equal(A.indptr, s.A.indptr) and np.array_equal(A.indices, s.A.indices)
    assert np.abs(A.data - s.A.data).max() <= 1e-13 * np.abs(s.A.data).max()
    info = dec.info()
    assert info.n_sub == odec.N
    for i in range(odec.N):
        dofs, pou, gn = dec.subdomain(i)
        assert np.array_equal(dofs, odec.dofs[i])
        assert np.abs(pou - odec.D[i]).max() <= 1e-15
        _, gnodes, _ = odec.G_local(i)
        assert np.array_equal(gn, gnodes)


@pytest.mark.parametrize("cfg", CASES)
def test_one_level_apply_matches_oracle(g, cfg):
    import torch
    from oracle import geneo as og
    geneo, ctx = g
    w = W.make(cfg)
    print("one-level", cfg, flush=True)
    sysm, dec = lib_problem(ctx, w)
    s, odec = oracle_problem(w)
    pc = ctx.setup(sysm, dec, coarse=geneo.COARSE_NONE)
    r = np.random.default_rng(3).standard_normal(s.n)
    z = torch.zeros(s.n, dtype=torch.float64, device="cuda:0")
    ctx.apply(pc, to_dev(r), z)
    torch.cuda.synchronize()
    zo = og.TwoLevel(odec, variant="as").apply(r)
    assert rel(z.cpu().numpy(), zo) <= solve_tol(odec)


@pytest.mark.parametrize("cfg", CASES)
def test_two_level_snk_apply_and_solve_match_oracle(g, cfg):
    import torch
    from oracle import geneo as og
    geneo, ctx = g
    w = W.make(cfg)
    print("snk", cfg, flush=True)
    sysm, dec = lib_problem(ctx, w)
    s, odec = oracle_problem(w)
    pc = ctx.setup(sysm, dec, coarse=geneo.COARSE_SNK)
    opc = og.TwoLevel(odec, variant="snk")
    info = pc.info()
    assert info.n0 == opc.n0 and info.n0_rank == opc.rank
    assert info.min_kept_pivot > 1e3 * max(info.max_dropped_pivot, 1e-300)
    r = np.random.default_rng(4).standard_normal(s.n)
    z = torch.zeros(s.n, dtype=torch.float64, device="cuda:0")
    ctx.apply(pc, to_dev(r), z)
    torch.cuda.synchronize()
    assert rel(z.cpu().numpy(), opc.apply(r)) <= 10 * solve_tol(odec)
    b = w.rhs(s.n)
    x = torch.zeros(s.n, dtype=torch.float64, device="cuda:0")
    si = ctx.solve(sysm, pc, to_dev(b), x, rtol=1e-8)
    xo, ito, _ = og.pcg(s.A, b, opc.apply, rtol=1e-8)
    xg = x.cpu().numpy()
    assert si.iterations == ito
    assert np.linalg.norm(b - s.A @ xg) <= 1.01e-8 * np.linalg.norm(b)
    assert rel(xg, xo) <= 1e-7


def test_solve_is_deterministic(g):
    import torch
    geneo, ctx = g
    w = W.make(1)
    sysm, dec = lib_problem(ctx, w)
    pc = ctx.setup(sysm, dec, coarse=geneo.COARSE_SNK)
    n = sysm.info().n
    b = to_dev(w.rhs(n))
    x1 = torch.zeros(n, dtype=torch.float64, device="cuda:0")
    x2 = torch.zeros_like(x1)
    i1 = ctx.solve(sysm, pc, b, x1)
    i2 = ctx.solve(sysm, pc, b, x2)
    assert i1.iterations == i2.iterations
    assert torch.equal(x1, x2)


@pytest.mark.parametrize("cfg,prec", [("1", "fp64"), ("small_channels", "fp64"), ("small_floating", "fp32")])
def test_pcg_graph_replays_match_eager(g, cfg, prec):
    """PCG with one iteration captured as a HIP graph and replayed (the
    library default) against kernel-by-kernel launches: same kernels in the
    same order, so the iterates are bitwise equal; every replay feeds the
    next, so a wrong replay would show in x.  Eager work on the context
    stream runs between two graph solves."""
    import torch
    geneo, ctx = g
    print("graph", cfg, prec, flush=True)
    w = W.make(int(cfg) if cfg.isdigit() else cfg)
    sysm, dec = lib_problem(ctx, w)
    lp = geneo.FP32_REFINE1 if prec == "fp32" else geneo.FP64
    pc = ctx.setup(sysm, dec, tau=w.tau, nev_max=w.nev_max, local_precision=lp)
    n = sysm.info().n
    rng = np.random.default_rng(11)
    for rep in range(2):
        b = to_dev(rng.standard_normal(n))
        xe = torch.zeros(n, dtype=torch.float64, device="cuda:0")
        xg = torch.full_like(xe, 7.0)
        ie = ctx.solve(sysm, pc, b, xe, rtol=1e-8, graph=False)
        z = torch.zeros_like(xe)
        ctx.apply(pc, b, z)   # eager work on the context stream between the solves
        ig = ctx.solve(sysm, pc, b, xg, rtol=1e-8, graph=True)
        torch.cuda.synchronize()
        assert ie.graph_replays == 0
        assert ig.iterations == ie.iterations
        assert ig.graph_replays == ig.iterations - 1 - ig.residual_replacements
        assert torch.equal(xe, xg)
        assert torch.isfinite(z).all()


def test_setup_on_reused_blocks_is_bitwise_identical(g):
    """The 24^3 channel workload's dense local, Neumann and coarse matrices
    (16-24 GB each) come back to the library's block pool when a
    preconditioner is freed; a second setup of the same problem runs on
    those reused blocks (holding the first setup's values) and must apply
    bitwise like the first."""
    import torch
    geneo, ctx = g
    print("pool reuse cube24", flush=True)
    w = W.make(2)
    sysm, dec = lib_problem(ctx, w)
    n = sysm.info().n
    r = to_dev(np.random.default_rng(12).standard_normal(n))
    z1 = torch.zeros(n, dtype=torch.float64, device="cuda:0")
    z2 = torch.zeros_like(z1)
    pc = ctx.setup(sysm, dec, tau=w.tau, nev_max=w.nev_max)
    ctx.apply(pc, r, z1)
    i1 = pc.info()
    torch.cuda.synchronize()
    del pc
    pc = ctx.setup(sysm, dec, tau=w.tau, nev_max=w.nev_max)
    ctx.apply(pc, r, z2)
    torch.cuda.synchronize()
    i2 = pc.info()
    assert (i1.n0, i1.n0_rank, i1.n_geneo) == (i2.n0, i2.n0_rank, i2.n_geneo)
    assert torch.equal(z1, z2)
    del pc


def test_pcg_maxit_exit_in_graph_mode(g):
    """PCG stopped by maxit: both launch modes report no convergence with the
    same 3 iterations and bitwise equal iterates, and a full solve on the
    same context afterwards (its stream restored) converges."""
    import torch
    geneo, ctx = g
    w = W.make(1)
    sysm, dec = lib_problem(ctx, w)
    pc = ctx.setup(sysm, dec, coarse=geneo.COARSE_SNK)
    n = sysm.info().n
    b = to_dev(w.rhs(n))
    xs = []
    for graph in (False, True):
        x = torch.zeros(n, dtype=torch.float64, device="cuda:0")
        si = ctx.solve(sysm, pc, b, x, rtol=1e-14, maxit=3, allow_noconv=True, graph=graph)
        assert si.iterations == 3 and si.rel_residual > 1e-14
        assert si.graph_replays == (2 if graph else 0)
        xs.append(x)
    torch.cuda.synchronize()
    assert torch.equal(xs[0], xs[1])
    x = torch.zeros(n, dtype=torch.float64, device="cuda:0")
    si = ctx.solve(sysm, pc, b, x, rtol=1e-8)
    torch.cuda.synchronize()
    assert si.rel_residual <= 1e-8
