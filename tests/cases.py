"""Shared helpers of the GPU tests: build the same workload in the library
and in the oracle (each from the seeded inputs only)."""
import numpy as np

import workloads as W


def lib_problem(ctx, w):
    sysm = ctx.assemble(w.mesh, w.mu, w.eps, w.gamma, w.dirichlet)
    p = w.partition
    if p["kind"] == "box":
        dec = ctx.partition(sysm, "box", box=p["p"], overlap=w.overlap)
    elif p["kind"] == "rcb":
        dec = ctx.partition(sysm, "rcb", nparts=p["nparts"], jitter=p["jitter"], overlap=w.overlap)
    else:
        dec = ctx.partition(sysm, "explicit", part_of_cell=p["part"], overlap=w.overlap)
    return sysm, dec


def oracle_problem(w):
    from oracle import decomp, fem
    s = fem.System(w.mesh, w.mu, w.eps, w.gamma, w.dirichlet)
    dec = decomp.Decomposition(s, decomp.partition_cells(w), w.overlap)
    return s, dec


def to_dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))


def solve_tol(dec, floor=1e-12):
    """Relative tolerance for comparing two FP64 results of dense Cholesky
    solves with the local matrices: their forward errors are bounded by
    about kappa(A_i) * unit roundoff each (backward-stable factorisation),
    so compare to 10 * eps * max_i kappa(A_i)."""
    kmax = max(np.linalg.cond(dec.A_dir(i).toarray()) for i in range(dec.N))
    return max(floor, 10 * np.finfo(float).eps * kmax)
