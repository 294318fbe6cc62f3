"""Benchmark of the AS-SNK-GenEO hot path on one MI355X.

A step is one pass of the whole path over one synthetic workload:
assemble, partition, setup (local Cholesky factors, GenEO eigenproblems,
coarse space and coarse Cholesky) and PCG to rtol 1e-8.  The default
workload is the full stack: a 128x16x16-hex beam (196,608 tets, h = 1/16)
with mu alternating 1 / 1e3 in 8 slabs along its length, eps = 1,
gamma = 1e-6, all-Dirichlet, 256 uneven subdomains by recursive coordinate
bisection with one overlap layer, at most 20 GenEO eigenvectors per
subdomain.  Two configurations run on the same mesh: the headline one with
FP32 local factors (conditioning check + probe + FP64 fallback) and the
learned warm start of the eigensolver, and the plain FP64 one with random
start blocks.  The model is trained beforehand (not timed) on other
instances of the same workload recipe.  The reported value is setup + solve
seconds with the assembled system already resident on the device; assembly
and partitioning are reported beside it.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                       [--variant both|learned_fp32|fp64] [--train-instances F]
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "setup+solve s to rtol 1e-8 & local-factor TFLOP/s; learned+FP32 vs plain FP64"
PEAK_FP64_TFLOPS = 78.6     # MI355X dense FP64 matrix peak
PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0       # MI355X HBM3E
# HBM bytes of one batched local factorisation per workload (plain FP64 path), from the
# rocprofv3 FETCH_SIZE and WRITE_SIZE counters summed over its launches and scaled by what the
# same counters read for a 1 GiB device copy (fetch x2.0, write x1.0); valid for the current
# potrf/trsm/syrk/mirror kernels only (a workload without a measurement reports null)
LOCAL_FACTOR_HBM_BYTES = {"cube24_channels": {"fetch": 193.9e9, "write": 57.2e9}}
# HBM bytes per coarse triangular-solve launch (the same counters, copy-scaled); none taken yet
COARSE_SOLVE_HBM_BYTES = {}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="5", help="workload id (default: the 128x16x16 slab beam)")
    ap.add_argument("--variant", default="both", choices=["both", "learned_fp32", "fp64"])
    ap.add_argument("--train-instances", type=int, default=8,
                    help="instances of the workload recipe the warm-start model is trained on (0: no model, the "
                         "learned_fp32 configuration then runs FP32 local factors with the cold start)")
    ap.add_argument("--coarse-order", default="auto", choices=["auto", "natural", "nd"],
                    help="elimination order of the coarse columns (nd: nested dissection of the subdomain graph; "
                         "auto: nested dissection where it shortens the coarse solves' dependency chain)")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the autotuner of the batched factorisation schedule (by default it times the "
                         "candidate schedules on matrices of the workload's local sizes before the timed steps)")
    ap.add_argument("--coarse-schedule", default="auto", choices=["auto", "steps", "levels"],
                    help="launch schedule of the coarse factorisation (levels: block columns of equal height in "
                         "its elimination tree together; auto: levels when the tree is at most half as tall as "
                         "the block column count)")
    ap.add_argument("--paper-table", default=None, choices=["gamma", "eps", "mu"],
                    help="instead of the benchmark: the paper's beam sweeps (Section 4, Numerical results: the "
                         "gamma sweep, alternating eps layers, alternating mu layers), one JSON line per case")
    ap.add_argument("--table-n", default="8,16", help="subdomain counts N of the paper-table beams")
    ap.add_argument("--table-cells", type=int, default=16, help="cells per unit length (the paper: 16)")
    ap.add_argument("--table-coarse", default="snk_geneo,snk",
                    help="coarse spaces of the paper-table runs (snk_geneo, snk, none, nk, nk_geneo)")
    ap.add_argument("--learned-study", default=None, metavar="TRAIN,HOLDOUT",
                    help="instead of the benchmark: train the warm-start model on TRAIN instances of workload 4 "
                         "(12^3-cell subdomains with random inclusions, gamma in [1e-6, 1]) and compare cold and "
                         "learned setups on HOLDOUT further instances; one JSON line")
    ap.add_argument("--study-epochs", type=int, default=30, help="training epochs of --learned-study")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run one device copy of BYTES (counter calibration) and exit")
    return ap.parse_args()


def partition(ctx, sysm, w):
    p = w.partition
    if p["kind"] == "box":
        return ctx.partition(sysm, "box", box=p["p"], overlap=w.overlap)
    return ctx.partition(sysm, "rcb", nparts=p["nparts"], jitter=p["jitter"], overlap=w.overlap)


def train_model(geneo, ctx, wid, n_inst):
    """Train the warm-start model on instances 1..n_inst of the workload
    recipe (the measured instance is instance 0); the last one is held out."""
    import workloads as W
    t0 = time.perf_counter()
    m = ctx.model_create(canvas=12, hidden=256, k=20, seed=2311)
    for f in range(1, n_inst + 1):
        w = W.make(wid, family=f)
        sysm = ctx.assemble(w.mesh, w.mu, w.eps, w.gamma, w.dirichlet)
        dec = partition(ctx, sysm, w)
        pc = ctx.setup(sysm, dec, tau=w.tau, nev_max=w.nev_max, keep_ritz=1)
        m.collect(sysm, dec, pc, holdout=(f == n_inst and n_inst > 1))
        del pc, dec, sysm
    t1 = time.perf_counter()
    ti = m.train(epochs=30, batch=32, lr=1e-3, seed=0)
    inf = m.info()
    return m, {"instances": n_inst, "samples_train": inf.n_train, "samples_holdout": inf.n_holdout,
               "params": inf.n_params, "data_s": t1 - t0, "train_ms": ti.train_ms,
               "loss_first_epoch": ti.loss_first, "loss_last_epoch": ti.loss_last, "holdout_loss": ti.holdout_loss}


def run_step(geneo, ctx, w, precision, b_host=None, model=None, coarse_order=0, coarse_schedule=0):
    import torch
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    t0 = time.perf_counter()
    sysm = ctx.assemble(w.mesh, w.mu, w.eps, w.gamma, w.dirichlet)
    t1 = time.perf_counter()
    dec = partition(ctx, sysm, w)
    n = sysm.info().n
    if b_host is None:
        b_host = w.rhs(n)
    b = torch.as_tensor(b_host, dtype=torch.float64, device="cuda:0")
    x = torch.zeros(n, dtype=torch.float64, device="cuda:0")
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    kw = {"model": model} if model is not None else {}
    pc = ctx.setup(sysm, dec, tau=w.tau, nev_max=w.nev_max, local_precision=precision, coarse_order=coarse_order,
                   coarse_schedule=coarse_schedule, **kw)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    si = ctx.solve(sysm, pc, b, x, rtol=1e-8, maxit=2000)
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    pi = pc.info()
    di = dec.info()
    out = dict(assemble_s=t1 - t0, partition_s=t2 - t1, setup_s=t3 - t2, solve_s=t4 - t3,
               setup_solve_s=t4 - t2, step_s=t4 - t0, iterations=si.iterations, rel_residual=si.rel_residual,
               true_rel_residual=si.true_rel_residual, residual_floor=si.residual_floor,
               graph_replays=si.graph_replays,
               n=n, n_sub=di.n_sub, n_min=di.n_min, n_max=di.n_max, n0=pi.n0, n0_rank=pi.n0_rank,
               n_snk=pi.n_snk, n_geneo=pi.n_geneo, lobpcg_iters=pi.lobpcg_iters,
               t_extract_ms=pi.t_extract_ms, t_factor_ms=pi.t_factor_ms, t_gevp_ms=pi.t_gevp_ms,
               t_coarse_build_ms=pi.t_coarse_build_ms, t_coarse_factor_ms=pi.t_coarse_factor_ms,
               t_coarse_refactor_ms=pi.t_coarse_refactor_ms,
               solve_ms=si.solve_ms, local_flops=pi.local_factor_flops, assemble_ms=sysm.info().assemble_ms,
               fp64_fallbacks=pi.fp64_fallbacks, fp32_rho_est=pi.fp32_rho_est,
               fp32_prechecked=pi.fp32_prechecked, fp32_kappa_lb=pi.fp32_kappa_lb,
               learned_starts=pi.learned_starts, start_residual=pi.start_residual,
               n0_factored=pi.n0 - pi.n0_local_dropped, coarse_flops=pi.coarse_factor_flops,
               coarse_fill=pi.coarse_fill, coarse_nd_levels=pi.coarse_nd_levels,
               coarse_solve_depth=pi.coarse_solve_depth, learned_candidates=pi.learned_candidates,
               lobpcg_unconverged=pi.lobpcg_unconverged, t_factor_fp32_ms=pi.t_factor_fp32_ms,
               coarse_lambda_min=pi.coarse_lambda_min, coarse_refactors=pi.coarse_refactors,
               coarse_drop_tol_used=pi.coarse_drop_tol_used, coarse_nd_predicted_depth=pi.coarse_nd_predicted_depth,
               coarse_solve_ms=si.coarse_solve_ms, coarse_solve_bytes=pi.coarse_solve_bytes,
               coarse_solves=si.coarse_solves, t_lobpcg_loop_ms=pi.t_lobpcg_loop_ms,
               coarse_levels=pi.coarse_levels, coarse_schedule=pi.coarse_schedule_used,
               lobpcg_solve_ms=pi.lobpcg_solve_ms, lobpcg_solve_bytes=pi.lobpcg_solve_bytes)
    del pc, dec, sysm
    return out, b_host


def cpu_baseline(w, budget_s=10.0, max_sample=32):
    """The oracle, as written, on a bounded sample of the same workload: the
    dense local Cholesky and the dense filtered GEVP (scipy eigh) of
    subdomains taken at evenly spaced quantiles of the subdomain sizes
    (smallest, largest, then the quantiles in between, bisected) until about
    `budget_s` seconds of oracle work, scaled by sum n_i^3 to all subdomains
    (the oracle's dense local work grows as n_i^3).  The coarse
    factorisation and the Krylov iteration are not in the sample: the
    oracle's coarse matrix (n0 ~ 1e5, dense) and a sparse direct solve of the
    whole system (223 s for the beam on 8 cores, SuperLU) exceed a bounded run."""
    from threadpoolctl import threadpool_info
    from oracle import decomp, fem, geneo
    import scipy.linalg as sla
    s = fem.System(w.mesh, w.mu, w.eps, w.gamma, w.dirichlet)
    dec = decomp.Decomposition(s, decomp.partition_cells(w), w.overlap)
    sizes = np.array([d.size for d in dec.dofs], dtype=np.float64)
    order = np.argsort(sizes, kind="stable")
    # quantile positions in bisection order: 0, 1, 1/2, 1/4, 3/4, 1/8, ...
    fr, k = [0.0, 1.0], 2
    while len(fr) < dec.N:
        fr += [(2 * j + 1) / k for j in range(k // 2)]
        k *= 2
    picks = []
    for f in fr:
        i = int(order[int(round(f * (dec.N - 1)))])
        if i not in picks:
            picks.append(i)
    t, sample = 0.0, []
    for i in picks[:max_sample]:
        Ai = dec.A_dir(i).toarray()
        Neu = dec.A_neu(i).toarray()
        Gi, _, _ = dec.G_local(i)
        t0 = time.perf_counter()
        sla.cholesky(Ai, lower=True)
        geneo.gevp(Ai, Neu, dec.D[i], Gi, w.tau, w.nev_max)
        t += time.perf_counter() - t0
        sample.append(i)
        if t >= budget_s:
            break
    scale = float((sizes ** 3).sum() / (sizes[sample] ** 3).sum())
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    return {"value": t * scale, "unit": "s", "cores": int(threads), "kind": "oracle",
            "sample": (f"dense local Cholesky + dense filtered GEVP (scipy eigh) of {len(sample)} subdomains at "
                       f"size quantiles (n_i {int(sizes[sample].min())} .. {int(sizes[sample].max())}) took "
                       f"{t:.1f} s, scaled by sum n_i^3 to all {dec.N} subdomains; coarse factor and Krylov "
                       "iteration excluded")}


def roof_gevp(plain):
    """The eigensolver against HBM: each LOBPCG iteration applies B^-1 (the
    local Neumann factors) to the k-column block, reading every factor's lower
    triangle once per sweep, sum n_j (n_j + 1) 8 bytes.  "achieved" is that
    over the HIP-event time of one application (both sweeps, the batched
    many-right-hand-side triangular solves); "loop_frac" is the same bytes
    times the iterations over the whole iteration loop (Gram products,
    Rayleigh-Ritz, the filtered-operator applies and the per-iteration
    convergence check included)."""
    sb = plain[-1]["lobpcg_solve_bytes"]
    sm = float(np.mean([r["lobpcg_solve_ms"] for r in plain]))
    lm = float(np.mean([r["t_lobpcg_loop_ms"] for r in plain]))
    its = plain[-1]["lobpcg_iters"]
    gbs = sb / (sm * 1e-3) / 1e9 if sm > 0 else None
    loop_gbs = sb * max(its - 1, 0) / (lm * 1e-3) / 1e9 if lm > 0 else None
    return {"bound": "hbm", "kernel": "batched B^-1 application in LOBPCG (k_trsm_multi_mfma, forward and "
                                      "backward sweeps over the local Neumann factors)",
            "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": gbs / PEAK_HBM_GBS if gbs else None, "bytes_per_application": sb,
            "ms_per_application": sm, "iterations": its, "loop_ms": lm,
            "loop_frac": loop_gbs / PEAK_HBM_GBS if loop_gbs else None, "traffic": None}


def summarize(res):
    mean = lambda k: float(np.mean([r[k] for r in res]))
    last = res[-1]
    return {
        "setup_solve_s": mean("setup_solve_s"),
        "setup_solve_steps_s": [r["setup_solve_s"] for r in res],
        "gevp_steps_ms": [r["t_gevp_ms"] for r in res],
        "local_factor_steps_ms": [r["t_factor_ms"] for r in res],
        "phases_ms": {"assemble": mean("assemble_s") * 1e3, "partition_host": mean("partition_s") * 1e3,
                      "setup": mean("setup_s") * 1e3, "solve": mean("solve_s") * 1e3,
                      "extract": mean("t_extract_ms"), "local_factor": mean("t_factor_ms"),
                      "gevp": mean("t_gevp_ms"), "coarse_build": mean("t_coarse_build_ms"),
                      "coarse_factor": mean("t_coarse_factor_ms"),
                      "coarse_refactor": mean("t_coarse_refactor_ms"), "pcg_device": mean("solve_ms")},
        "local_factor_tflops": last["local_flops"] / (mean("t_factor_ms") * 1e-3) / 1e12,
        "fp32_factor_ms": mean("t_factor_fp32_ms"),
        # FP32 factorisation rate: only when every subdomain went through it (none routed to FP64
        # by the conditioning check before the FP32 factorisation)
        "fp32_factor_tflops": (last["local_flops"] / (mean("t_factor_fp32_ms") * 1e-3) / 1e12
                               if mean("t_factor_fp32_ms") > 0 and last["fp32_prechecked"] == 0 else None),
        "coarse_factor_tflops": last["coarse_flops"] / (mean("t_coarse_factor_ms") * 1e-3) / 1e12,
        "coarse_fill": last["coarse_fill"], "coarse_nd_levels": last["coarse_nd_levels"],
        "coarse_solve_depth": last["coarse_solve_depth"], "lobpcg_unconverged": last["lobpcg_unconverged"],
        "coarse_nd_predicted_depth": last["coarse_nd_predicted_depth"], "coarse_lambda_min": last["coarse_lambda_min"],
        "coarse_refactors": last["coarse_refactors"], "coarse_drop_tol_used": last["coarse_drop_tol_used"],
        "coarse_solve_ms": mean("coarse_solve_ms"), "coarse_solve_bytes": last["coarse_solve_bytes"],
        "coarse_solves": last["coarse_solves"], "lobpcg_loop_ms": mean("t_lobpcg_loop_ms"),
        "coarse_levels": last["coarse_levels"],
        "coarse_schedule": {1: "steps", 2: "levels"}.get(last["coarse_schedule"], "steps"),
        "lobpcg_solve_ms": mean("lobpcg_solve_ms"),
        "learned_candidates": last["learned_candidates"],
        "pcg_iterations": last["iterations"], "rel_residual": last["rel_residual"],
        "true_rel_residual": last["true_rel_residual"], "residual_floor": last["residual_floor"],
        "pcg_graph_replays": last["graph_replays"],
        "lobpcg_iterations": last["lobpcg_iters"], "start_residual": last["start_residual"],
        "learned_starts": last["learned_starts"], "fp64_fallbacks": last["fp64_fallbacks"],
        "fp32_rho_est": last["fp32_rho_est"] if np.isfinite(last["fp32_rho_est"]) else "inf",
        "fp32_prechecked": last["fp32_prechecked"],
        "fp32_kappa_lb": last["fp32_kappa_lb"] if np.isfinite(last["fp32_kappa_lb"]) else "inf",
    }


def copy_calibration(nbytes):
    """One device-to-device copy of nbytes: the reference kernel for scaling
    the FETCH_SIZE / WRITE_SIZE counters of the hot path to bytes."""
    import torch
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": a.numel() * 8}), flush=True)


def paper_tables(a):
    """The paper's beam sweeps on the GPU: for each case, AS with the chosen
    coarse spaces, right-preconditioned GMRES to 1e-6 (the paper's solver and
    tolerance) and PCG to 1e-8; one JSON line per (case, coarse space) with
    the iteration counts and the coarse space sizes."""
    import torch
    from paper_2311_18783_amd import geneo
    import workloads as W
    kinds = {"snk_geneo": geneo.COARSE_SNK_GENEO, "snk": geneo.COARSE_SNK, "none": geneo.COARSE_NONE,
             "nk": geneo.COARSE_NK, "nk_geneo": geneo.COARSE_NK_GENEO}
    if a.paper_table == "gamma":
        cases = [dict(gamma=g, bc="all") for g in (1e-5, 1e-4, 1e-3, 1e-2, 1e-1, 1.0, 10.0, 100.0)]
    else:
        cases = [dict(gamma=1e-3, bc=bc, layers=a.paper_table, alt=v)
                 for bc in ("all", "mixed") for v in (1e-4, 1e-3, 1e-2, 1e-1, 1.0, 10.0, 1e2, 1e3, 1e4)]
    ctx = geneo.Context(0)
    for N in [int(x) for x in a.table_n.split(",")]:
        for c in cases:
            w = W.paper_beam(N, cells=a.table_cells, **c)
            sysm = ctx.assemble(w.mesh, w.mu, w.eps, w.gamma, w.dirichlet)
            dec = ctx.partition(sysm, "box", box=w.partition["p"], overlap=w.overlap)
            n = sysm.info().n
            b = torch.as_tensor(w.rhs(n), device="cuda:0")
            for kname in a.table_coarse.split(","):
                pc = ctx.setup(sysm, dec, tau=w.tau, nev_max=w.nev_max, coarse=kinds[kname])
                pi = pc.info()
                row = {"table": a.paper_table, "N": N, "cells": a.table_cells, **c, "coarse": kname, "n": n,
                       "n_snk": pi.n_snk, "n_geneo": pi.n_geneo, "n0_rank": pi.n0_rank,
                       "lobpcg_unconverged": pi.lobpcg_unconverged}
                for meth, rtol, key in ((geneo.GMRES, 1e-6, "gmres_1e-6"), (geneo.PCG, 1e-8, "pcg_1e-8")):
                    x = torch.zeros(n, dtype=torch.float64, device="cuda:0")
                    si = ctx.solve(sysm, pc, b, x, rtol=rtol, maxit=500, method=meth, allow_noconv=True)
                    row[key] = si.iterations if si.rel_residual <= rtol else None
                print(json.dumps(row), flush=True)
                del pc
            del dec, sysm
    ctx.close()


def learned_study(a):
    """Learned warm start on workload 4: the model is trained on GEVP solutions
    of TRAIN instances (the cold eigensolver's Ritz vectors), its loss checked
    on HOLDOUT other instances, and the eigensolver run on those HOLDOUT
    instances from the cold start and from the judged learned start."""
    from paper_2311_18783_amd import geneo
    import workloads as W
    n_train, n_hold = (int(x) for x in a.learned_study.split(","))
    ctx = geneo.Context(0)
    m = ctx.model_create(canvas=12, hidden=256, k=20, seed=2311)
    t0 = time.perf_counter()
    for f in range(1, n_train + n_hold + 1):
        w = W.make(4, family=f)
        sysm = ctx.assemble(w.mesh, w.mu, w.eps, w.gamma, w.dirichlet)
        dec = partition(ctx, sysm, w)
        pc = ctx.setup(sysm, dec, tau=w.tau, nev_max=w.nev_max, keep_ritz=1)
        m.collect(sysm, dec, pc, holdout=f > n_train)
        del pc, dec, sysm
        if f % 25 == 0:
            print(f"[learned-study] collected {f} instances, {time.perf_counter() - t0:.0f} s", file=sys.stderr,
                  flush=True)
    t1 = time.perf_counter()
    ti = m.train(epochs=a.study_epochs, batch=32, lr=1e-3, seed=0)
    inf = m.info()
    rows = []
    for f in range(n_train + 1, n_train + n_hold + 1):
        w = W.make(4, family=f)
        sysm = ctx.assemble(w.mesh, w.mu, w.eps, w.gamma, w.dirichlet)
        dec = partition(ctx, sysm, w)
        r = {"gamma": w.gamma}
        for tag, kw in (("cold", {}), ("learned", {"model": m})):
            pc = ctx.setup(sysm, dec, tau=w.tau, nev_max=w.nev_max, **kw)
            pi = pc.info()
            r[tag] = {"lobpcg_iterations": pi.lobpcg_iters, "gevp_ms": pi.t_gevp_ms,
                      "unconverged": pi.lobpcg_unconverged, "n_geneo": pi.n_geneo,
                      "learned_starts": pi.learned_starts, "start_residual": pi.start_residual}
            del pc
        rows.append(r)
        del dec, sysm
    mean = lambda tag, k: float(np.mean([r[tag][k] for r in rows]))
    line = {"study": "learned warm start, workload 4", "train_instances": n_train, "holdout_instances": n_hold,
            "samples_train": inf.n_train, "samples_holdout": inf.n_holdout, "params": inf.n_params,
            "data_s": t1 - t0, "train_ms": ti.train_ms, "epochs": a.study_epochs,
            "loss_first_epoch": ti.loss_first, "loss_last_epoch": ti.loss_last, "holdout_loss": ti.holdout_loss,
            "loss_of_a_zero_prediction": 20,
            "cold": {k: mean("cold", k) for k in ("lobpcg_iterations", "gevp_ms", "start_residual")},
            "learned": {k: mean("learned", k) for k in ("lobpcg_iterations", "gevp_ms", "start_residual",
                                                          "learned_starts")},
            "per_instance": rows}
    print(json.dumps(line), flush=True)
    ctx.close()


def main():
    a = parse()
    if a.learned_study:
        learned_study(a)
        return
    if a.copy_calibration:
        copy_calibration(a.copy_calibration)
        return
    if a.paper_table:
        paper_tables(a)
        return
    if a.gpus != 1:
        print(json.dumps({"error": "single-GPU benchmark: the batched per-subdomain work runs on one GPU; "
                                   "--gpus must be 1", "n_gpus": a.gpus}))
        sys.exit(2)
    import torch
    from paper_2311_18783_amd import geneo
    import workloads as W
    wid = int(a.workload) if a.workload.isdigit() else a.workload
    w = W.make(wid)
    ctx = geneo.Context(0)
    variants = {"learned_fp32": (geneo.FP32_REFINE1, True), "fp64": (geneo.FP64, False)}
    run = [v for v in ("learned_fp32", "fp64") if a.variant in ("both", v)]
    model, training = None, None
    corder = {"nd": geneo.ORDER_NESTED_DISSECTION, "natural": geneo.ORDER_NATURAL, "auto": geneo.ORDER_AUTO}[a.coarse_order]
    csched = {"auto": geneo.SCHEDULE_AUTO, "steps": geneo.SCHEDULE_STEPS,
              "levels": geneo.SCHEDULE_LEVELS}[a.coarse_schedule]
    schedules = None
    if not a.no_tune:
        # the local (and Neumann) matrix sizes of this workload's decomposition
        sysm = ctx.assemble(w.mesh, w.mu, w.eps, w.gamma, w.dirichlet)
        dec = partition(ctx, sysm, w)
        sizes = [len(dec.subdomain(i)[0]) for i in range(dec.info().n_sub)]
        del dec, sysm
        schedules = {}
        for v in run:
            prec = variants[v][0]
            mode, group, potrf, ms, tried = ctx.tune_factor(sizes, prec, reps=2)
            schedules["fp32" if prec == geneo.FP32_REFINE1 else "fp64"] = {
                "mode": mode, "group": group, "potrf": potrf, "ms": ms, "candidates": tried}
    if "learned_fp32" in run and a.train_instances > 0:
        model, training = train_model(geneo, ctx, wid, a.train_instances)
    b_host = None
    for _ in range(a.warmup):
        for v in run:
            prec, learned = variants[v]
            _, b_host = run_step(geneo, ctx, w, prec, b_host, model if learned else None, corder, csched)
    torch.cuda.synchronize()
    res = {v: [] for v in run}
    t0 = time.perf_counter()
    for _ in range(a.steps):
        for v in run:
            prec, learned = variants[v]
            r, b_host = run_step(geneo, ctx, w, prec, b_host, model if learned else None, corder, csched)
            res[v].append(r)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    summ = {v: summarize(res[v]) for v in run}
    head = run[0]
    last = res[head][-1]
    plain = res["fp64"] if "fp64" in res else res[head]
    # The two candidate dominant kernels, on the plain FP64 path: the batched local Cholesky
    # (sum n_i^3 / 3 flop over the HIP-event time of the factorisation of all subdomain
    # matrices) and the coarse triangular solves (k_trsv: every tile of the factor's pattern
    # read once per sweep, over the HIP-event time of the first two solves, times the number of
    # solves PCG ran).  "roofline" is the one with the larger device time per step; the coarse
    # factorisation and the eigensolver's B^-1 application beside them.
    lf_ms = float(np.mean([r["t_factor_ms"] for r in plain]))
    achieved = plain[-1]["local_flops"] / (lf_ms * 1e-3) / 1e12
    cf_ms = float(np.mean([r["t_coarse_factor_ms"] for r in plain]))
    # flops of the coarse factorisation as performed: on the block-sparse fill pattern of E
    achieved_coarse = plain[-1]["coarse_flops"] / (cf_ms * 1e-3) / 1e12
    cs_ms = float(np.mean([r["coarse_solve_ms"] for r in plain]))
    cs_bytes = plain[-1]["coarse_solve_bytes"]
    cs_step_ms = cs_ms * plain[-1]["coarse_solves"]
    roof_local = {"bound": "mfma",
                  "kernel": f"batched FP64 local Cholesky of the {last['n_sub']} subdomain matrices "
                            "(potrf/trsm/syrk/mirror)",
                  "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                  "frac": achieved / PEAK_FP64_TFLOPS,
                  "traffic": (sum(LOCAL_FACTOR_HBM_BYTES[w.name].values())
                              if w.name in LOCAL_FACTOR_HBM_BYTES else None),
                  "traffic_unit": "B per factorisation (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled)",
                  "ms_per_step": lf_ms}
    cs_gbs = (cs_bytes / 2) / (cs_ms / 2 * 1e-3) / 1e9 if cs_ms > 0 else None
    roof_solve = {"bound": "hbm",
                  "kernel": "coarse block triangular solves (k_trsv, forward and backward sweeps over the "
                            "factor's tiles)",
                  "achieved": cs_gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                  "frac": cs_gbs / PEAK_HBM_GBS if cs_gbs else None,
                  "bytes_per_launch": cs_bytes / 2, "ms_per_launch": cs_ms / 2,
                  "traffic": COARSE_SOLVE_HBM_BYTES.get(w.name), "traffic_unit": "B per launch (copy-scaled)",
                  "ms_per_step": cs_step_ms}
    solve_dominant = cs_step_ms > lf_ms
    line = {
        "metric": METRIC,
        "value": summ[head]["setup_solve_s"],
        "unit": "s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": wall / (a.steps * len(run)) * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.describe}, tau = {w.tau:g}, <= {w.nev_max} GenEO vectors "
                               "per subdomain, PCG rtol 1e-8",
                   "variant": head, "n": last["n"], "n_sub": last["n_sub"], "n_i_min": last["n_min"],
                   "n_i_max": last["n_max"], "n0": last["n0"], "n0_factored": last["n0_factored"],
                   "n0_rank": last["n0_rank"],
                   "n_geneo": last["n_geneo"], "parallelism": "1 GPU"},
        "variants": summ,
        "roofline": roof_solve if solve_dominant else roof_local,
        ("roofline_local_factor" if solve_dominant else "roofline_coarse_solve"):
            roof_local if solve_dominant else roof_solve,
        "roofline_coarse": {"bound": "mfma", "kernel": "block-sparse FP64 coarse Cholesky of E",
                            "achieved": achieved_coarse, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                            "frac": achieved_coarse / PEAK_FP64_TFLOPS},
        "roofline_gevp": roof_gevp(plain),
    }
    if "fp64" in summ and head != "fp64":
        line["speedup_vs_plain_fp64"] = summ["fp64"]["setup_solve_s"] / summ[head]["setup_solve_s"]
    if training:
        line["warm_start_training"] = training
    if schedules:
        line["factor_schedules"] = schedules
    if not a.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
