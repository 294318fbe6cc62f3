"""GPU: FP32 local factors with one FP64 refinement step, the probe of
rho(I - Ahat_i^-1 A_i) and the per-subdomain FP64 fallback."""
import numpy as np
import pytest

import workloads as W
from cases import lib_problem, oracle_problem, rel, to_dev

pytestmark = pytest.mark.gpu

CASES = ["1", "small_mixed", "small_floating", "small_hole", "small_channels"]


@pytest.fixture(scope="module")
def g():
    import torch
    from paper_2311_18783_amd import geneo
    assert torch.cuda.is_available()
    ctx = geneo.Context(0)
    yield geneo, ctx
    ctx.close()


def _rho_oracle(w):
    """Exact spectral radii of I - Ahat_i^-1 A_i with LAPACK's FP32 factors."""
    from oracle import geneo as og
    s, odec = oracle_problem(w)
    tl = og.TwoLevel(odec, variant="as", local_precision="fp32_refine1")
    return s, np.array([tl.fp32_rho(i) for i in range(odec.N)]), tl


def _scaled_kappa(w):
    """Condition numbers of D^-1/2 A_i D^-1/2 (D = diag A_i), dense eigenvalues."""
    s, odec = oracle_problem(w)
    out = []
    for d in odec.dofs:
        Ai = s.A[d][:, d].toarray()
        r = 1.0 / np.sqrt(np.diag(Ai))
        ev = np.linalg.eigvalsh(Ai * r[:, None] * r[None, :])
        out.append(ev[-1] / ev[0])
    return np.array(out)


@pytest.mark.parametrize("cfg", CASES)
def test_fp32_refined_preconditioner(g, cfg):
    """Fallback count consistent with the exact radii (every subdomain with
    rho > 1 falls back, none with rho < 0.25 does unless fewer than 1 in 8
    subdomains would keep FP32, when all do); the FP32 apply differs
    from the FP64 apply by O(rho^2) (the refined local error); PCG stays
    within one iteration of FP64 and reaches rtol 1e-8."""
    import torch
    geneo, ctx = g
    print("fp32", cfg, flush=True)
    w = W.make(int(cfg) if cfg.isdigit() else cfg)
    s, rho, tl = _rho_oracle(w)
    sysm, dec = lib_problem(ctx, w)
    pc64 = ctx.setup(sysm, dec, tau=w.tau, nev_max=w.nev_max, local_precision=geneo.FP64)
    pc32 = ctx.setup(sysm, dec, tau=w.tau, nev_max=w.nev_max, local_precision=geneo.FP32_REFINE1)
    i64, i32 = pc64.info(), pc32.info()
    assert i32.n0 == i64.n0 and i32.n_geneo == i64.n_geneo and i32.n0_rank == i64.n0_rank
    nfb = i32.fp64_fallbacks
    N = rho.size
    assert int((rho > 1.0).sum()) <= nfb, (nfb, rho)
    # every subdomain with rho < 0.25 keeps FP32 unless fewer than 1 in 8 would (then all go to FP64)
    assert nfb <= int((rho > 0.25).sum()) or (nfb == N and 8 * int((rho <= 0.25).sum()) < N), (nfb, rho)
    # the conditioning check only skips subdomains whose FP32 factor the probe rejects,
    # and its bound is a lower bound of the scaled condition number
    assert i32.fp32_prechecked <= int((rho > 0.5).sum()), (i32.fp32_prechecked, rho)
    assert 0 < i32.fp32_kappa_lb <= (1 + 1e-6) * _scaled_kappa(w).max()
    assert i32.fp32_rho_est > 0
    if nfb == 0:
        assert i32.fp32_rho_est <= 0.5
        assert 0.1 * rho.max() <= i32.fp32_rho_est <= 10 * rho.max(), (i32.fp32_rho_est, rho.max())
    r = np.random.default_rng(5).standard_normal(s.n)
    z64 = torch.zeros(s.n, dtype=torch.float64, device="cuda:0")
    z32 = torch.zeros_like(z64)
    ctx.apply(pc64, to_dev(r), z64)
    ctx.apply(pc32, to_dev(r), z32)
    torch.cuda.synchronize()
    rmax = min(0.5, float(rho[rho <= 0.5].max())) if (rho <= 0.5).any() else 0.0
    tol = 10 * rmax ** 2 + 1e-10
    assert rel(z32.cpu().numpy(), z64.cpu().numpy()) <= tol
    if nfb == 0:
        # one-level FP32 apply against the oracle's (LAPACK FP32 factors, one FP64 refinement
        # step): each refined local solve is within rho^2 of A_i^-1 R_i r
        pcn = ctx.setup(sysm, dec, coarse=geneo.COARSE_NONE, local_precision=geneo.FP32_REFINE1)
        assert pcn.info().fp64_fallbacks == 0
        zn = torch.zeros(s.n, dtype=torch.float64, device="cuda:0")
        ctx.apply(pcn, to_dev(r), zn)
        torch.cuda.synchronize()
        e = rel(zn.cpu().numpy(), tl.one_level(r))
        print("fp32 one-level vs oracle", cfg, e, "rho max", rho.max(), flush=True)
        assert e <= 10 * rho.max() ** 2 + 1e-10
    b = w.rhs(s.n)
    x64 = torch.zeros(s.n, dtype=torch.float64, device="cuda:0")
    x32 = torch.zeros_like(x64)
    s64 = ctx.solve(sysm, pc64, to_dev(b), x64, rtol=1e-8)
    s32 = ctx.solve(sysm, pc32, to_dev(b), x32, rtol=1e-8)
    assert s32.iterations <= s64.iterations + 1, (s32.iterations, s64.iterations)
    xg = x32.cpu().numpy()
    assert np.linalg.norm(b - s.A @ xg) <= 1.01e-8 * np.linalg.norm(b)


def test_fp32_full_fallback_is_the_fp64_path(g):
    """fp32_rho_max = 0 sends every subdomain to FP64: the apply is then
    bitwise that of the FP64 preconditioner."""
    import torch
    geneo, ctx = g
    w = W.make("small_floating")
    sysm, dec = lib_problem(ctx, w)
    n = sysm.info().n
    pc64 = ctx.setup(sysm, dec, tau=w.tau, nev_max=w.nev_max, local_precision=geneo.FP64)
    pcf = ctx.setup(sysm, dec, tau=w.tau, nev_max=w.nev_max, local_precision=geneo.FP32_REFINE1,
                    fp32_rho_max=0.0)
    assert pcf.info().fp64_fallbacks == dec.info().n_sub
    r = to_dev(np.random.default_rng(6).standard_normal(n))
    a = torch.zeros(n, dtype=torch.float64, device="cuda:0")
    b = torch.zeros_like(a)
    ctx.apply(pc64, r, a)
    ctx.apply(pcf, r, b)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_fp32_conditioning_check_skips_hopeless_factors(g):
    """With gamma = 1e-6 every local matrix of the channel case is too ill
    conditioned for an FP32 factor (LAPACK's fails or its refinement radius
    exceeds 0.5): the conditioning check sends all of them to FP64 before
    any FP32 work, its bound stays below the scaled condition numbers, and
    the apply is bitwise that of the FP64 preconditioner."""
    import scipy.linalg as sla
    import torch
    geneo, ctx = g
    w = W.make("small_channels", gamma=1e-6)
    s, odec = oracle_problem(w)
    for d in odec.dofs:
        Ai = s.A[d][:, d].toarray()
        try:
            L = sla.cholesky(Ai.astype(np.float32), lower=True).astype(np.float64)
        except np.linalg.LinAlgError:
            continue
        T = np.eye(len(d)) - sla.cho_solve((L, True), Ai)
        assert np.abs(np.linalg.eigvals(T)).max() > 0.5
    sysm, dec = lib_problem(ctx, w)
    n = sysm.info().n
    pc64 = ctx.setup(sysm, dec, tau=w.tau, nev_max=w.nev_max, local_precision=geneo.FP64)
    pc32 = ctx.setup(sysm, dec, tau=w.tau, nev_max=w.nev_max, local_precision=geneo.FP32_REFINE1)
    i32 = pc32.info()
    assert i32.fp32_prechecked == dec.info().n_sub
    assert i32.fp64_fallbacks == dec.info().n_sub
    assert 0.2 * 2.0 ** -24 * i32.fp32_kappa_lb > 0.5
    assert i32.fp32_kappa_lb <= (1 + 1e-6) * _scaled_kappa(w).max()
    r = to_dev(np.random.default_rng(7).standard_normal(n))
    a = torch.zeros(n, dtype=torch.float64, device="cuda:0")
    b = torch.zeros_like(a)
    ctx.apply(pc64, r, a)
    ctx.apply(pc32, r, b)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
