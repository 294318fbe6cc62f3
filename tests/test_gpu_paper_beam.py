"""GPU: the paper's weak-scaling beam (Section 4 "Numerical results", influence of the geometry):
N/2 x 1 x 1 with h = 1/16, N strip subdomains, one overlap layer,
mu = eps = 1, gamma = 1e-3.  The paper reports, for AS-SNK-GenEO on the
homogeneous beam, iteration counts that stay nearly constant as N grows
(Dirichlet and mixed boundary conditions) and an empty GenEO part with
Dirichlet conditions on every face; here the mixed beam's GenEO part holds
one column per interior strip (the harmonic field grad z of a strip whose
Dirichlet boundary has two components; pinned on the CPU).  At h = 1/8 and
N = 8 the library matches the oracle on the paper's sweeps (gamma,
alternating eps and mu layers): GenEO sizes, coarse rank and GMRES
iteration counts to 1e-6 (the paper's solver and tolerance)."""
import numpy as np
import pytest

import workloads as W
from cases import lib_problem, oracle_problem, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def g():
    import torch
    from paper_2311_18783_amd import geneo
    assert torch.cuda.is_available()
    ctx = geneo.Context(0)
    yield geneo, ctx
    ctx.close()


def _run(g, N, rule):
    import torch
    geneo, ctx = g
    print("beam", N, rule, flush=True)
    w = W.make(f"beam{N}")
    w.dirichlet = W.dirichlet_flags(w.mesh["bface_tag"], rule)
    sysm, dec = lib_problem(ctx, w)
    pc = ctx.setup(sysm, dec, tau=w.tau, nev_max=w.nev_max)
    n = sysm.info().n
    x = torch.zeros(n, dtype=torch.float64, device="cuda:0")
    si = ctx.solve(sysm, pc, to_dev(w.rhs(n)), x, rtol=1e-8)
    info = pc.info()
    del pc
    assert si.rel_residual <= 1e-8
    return si.iterations, info.n_geneo


@pytest.mark.parametrize("rule", ["all", "mixed"])
def test_beam_weak_scaling_iterations_stay_flat(g, rule):
    it8, gen8 = _run(g, 8, rule)
    it16, gen16 = _run(g, 16, rule)
    print(rule, "iterations", it8, it16, "GenEO", gen8, gen16, flush=True)
    assert it16 <= it8 + 3
    if rule == "all":
        assert gen8 == 0 and gen16 == 0
    else:
        assert gen8 == 8 - 2 and gen16 == 16 - 2


@pytest.mark.parametrize("case", [dict(gamma=1e-3, bc="all"), dict(gamma=1e-5, bc="all"),
                                  dict(gamma=1e-3, bc="mixed", layers="mu", alt=1e4),
                                  dict(gamma=1e-3, bc="mixed", layers="eps", alt=1e-4)],
                         ids=["gamma1e-3", "gamma1e-5", "mu1e4_mixed", "eps1e-4_mixed"])
def test_paper_beam_h8_matches_oracle(g, case):
    """N = 8 strips at h = 1/8 (32 x 8 x 8 hexes): the GenEO size, the
    coarse size and rank equal the oracle's, and right-preconditioned GMRES
    to 1e-6 needs as many iterations as the oracle's GMRES with the oracle's
    preconditioner."""
    import torch
    from oracle import geneo as og
    geneo, ctx = g
    w = W.paper_beam(8, cells=8, **case)
    print("paper beam h = 1/8", w.name, flush=True)
    s, odec = oracle_problem(w)
    opc = og.TwoLevel(odec, tau=w.tau, nev_max=w.nev_max)
    sysm, dec = lib_problem(ctx, w)
    pc = ctx.setup(sysm, dec, tau=w.tau, nev_max=w.nev_max)
    info = pc.info()
    assert info.n_geneo == opc.n_geneo and info.n0 == opc.n0 and info.n0_rank == opc.rank, \
        (info.n_geneo, opc.n_geneo, info.n0, opc.n0, info.n0_rank, opc.rank)
    b = w.rhs(s.n)
    x = torch.zeros(s.n, dtype=torch.float64, device="cuda:0")
    si = ctx.solve(sysm, pc, to_dev(b), x, rtol=1e-6, method=geneo.GMRES)
    _, ito, _ = og.gmres(s.A, b, opc.apply, rtol=1e-6)
    print("GenEO", info.n_geneo, "GMRES iterations", si.iterations, "oracle", ito, flush=True)
    assert si.iterations == ito
    xg = x.cpu().numpy()
    assert np.linalg.norm(b - s.A @ xg) <= 1.01e-6 * np.linalg.norm(b)
