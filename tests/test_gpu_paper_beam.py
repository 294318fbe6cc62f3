"""GPU: the paper's weak-scaling beam (Section 4 "Numerical results", influence of the geometry):
N/2 x 1 x 1 with h = 1/16, N strip subdomains, one overlap layer,
mu = eps = 1, gamma = 1e-3.  The paper reports, for AS-SNK-GenEO on the
homogeneous beam, iteration counts that stay nearly constant as N grows
(Dirichlet and mixed boundary conditions) and an empty GenEO part with
Dirichlet conditions on every face.  Qualitative check only: the paper
uses right-preconditioned GMRES to 1e-6 on FreeFEM meshes, here PCG to 1e-8."""
import pytest

import workloads as W
from cases import lib_problem, to_dev

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
