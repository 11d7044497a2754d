"""Measurements of the configurations other than the benchmark's default
(bench.py --workload fp64|batch|diff).  Each returns one JSON-able dict.

* fp64:  8x8x1 grid, 112 interfaces, n~U{200..400}, complex128 factor and
         solve, 1 and 16 right-hand sides (the plain method).
* batch: a frequency sweep of 32 instances (grids 2x2x2 / 3x3x2 / 4x4x2,
         n~U{100..500}, f in [0.5, 2]), 16 RHS each, complex64 + FP64
         refinement, one persistent launch per phase, captured in a hipGraph
         and replayed; plan knobs tuned on the batch as a whole.
* pivot: the precision workload (4x4x4) factored with Bunch-Kaufman pivoting
         inside each diagonal tile, both precisions, against the unpivoted
         factor on the same K.
* primal: primal reduction (interior blocks of a 4x4x4 domain grid
         eliminated onto the interfaces), the reduced system's mixed
         solve, and the primal recovery with 8 port projections.
* diff:  6x6x6 grid, 540 interfaces, n~U{300..700} (about 270k unknowns),
         128 RHS, complex64 + FP64 refinement, then the adjoint (lambda and
         dK on K's pattern) with the same factors.  Its gradient is checked
         against the CPU FP64 reference on a sub-instance in the GPU tests.
"""
from __future__ import annotations

import json
import sys
import time

import numpy as np

PEAK_FP32_MFMA = 157.3
PEAK_FP64_MFMA = 78.6


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _events():
    import torch
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def fp64(args):
    import torch

    import paper_2002_05026_amd as d3m
    from paper_2002_05026_amd import instances as gen
    res = {"metric": "block-LDLT TFLOP/s + time-to-solve, FP64 plain method", "unit": "TFLOP/s",
           "data": "synthetic", "dtype": "c128", "n_gpus": 1,
           "config": {"workload": "fp64: 8x8x1 domain grid, 112 interfaces, n~U{200..400}, complex128"}}
    from paper_2002_05026_amd import tune
    runs = {}
    for nrhs in (int(v) for v in str(getattr(args, "fp64_nrhs", "1,16")).split(",")):
        inst = gen.config_fp64(nrhs=nrhs)
        if getattr(args, "knobs", None):
            kn = json.loads(args.knobs)
            kn = kn.get("c128", kn) if ("c64" in kn or "c128" in kn) else kn
            tuned = {"config": dict(tune.DEFAULT, **kn)}
        elif getattr(args, "no_tune", False):
            tuned = {"config": dict(tune.DEFAULT)}
        else:
            tuned = tune.tune(inst, d3m.C128, nrhs=nrhs, reps=2, save=False)
        _log(f"fp64 nrhs={nrhs} tuned {tuned}")
        plan = d3m.Plan(inst.sizes, inst.pairs, grid=inst.grid, **tuned["config"])
        flops = plan.info["flops_factor"]
        K = torch.from_numpy(inst.K).cuda()
        B = torch.from_numpy(inst.B).cuda()
        X = torch.empty_like(B)
        f = d3m.Factor(plan, d3m.C128, nrhs_max=nrhs, timing=True)
        for _ in range(max(1, args.warmup)):
            f.factorize(K)
            f.solve(B, X)
        torch.cuda.synchronize()
        f.status()
        e0, e1 = _events()
        e0.record()
        for _ in range(args.steps):
            f.factorize(K)
            f.solve(B, X)
        e1.record()
        torch.cuda.synchronize()
        st = f.status()
        ms = e0.elapsed_time(e1) / args.steps
        dag = st["t_factor_dag_ms"] / st["n_factor_dag"]
        sdag = st["t_solve_dag_ms"] / st["n_solve_dag"]
        solve_bytes = 2.0 * plan.info["nnz_L"] * 16
        runs[nrhs] = {"N": inst.N, "time_to_solve_ms": ms, "factor_dag_ms": dag, "factor_tflops": flops / dag / 1e9,
                      "frac_fp64_peak": flops / dag / 1e9 / PEAK_FP64_MFMA, "solve_dag_ms": sdag,
                      "solve_GBps_factor_bytes": solve_bytes / sdag / 1e6, "eta": st["eta"],
                      "factor_gflop": flops / 1e9, "tuned": tuned["config"]}
        _log(f"fp64 nrhs={nrhs}: {runs[nrhs]}")
    res["runs"] = runs
    res["value"] = runs[min(runs)]["factor_tflops"]
    return res


def batch(args):
    import torch

    import paper_2002_05026_amd as d3m
    from paper_2002_05026_amd import instances as gen
    from paper_2002_05026_amd import tune
    insts = gen.config_batch(count=32, nrhs=16)
    _log(f"batch: {len(insts)} instances, N = {[i.N for i in insts][:8]}...")
    Ks = [torch.from_numpy(inst.K).cuda() for inst in insts]
    Bs = [torch.from_numpy(inst.B).cuda() for inst in insts]
    # plan knobs tuned on the batch itself (each candidate timed as a whole
    # merged run), outside the timed region
    if getattr(args, "knobs", None):
        kn = json.loads(args.knobs)
        kn = kn.get("c64", kn) if ("c64" in kn or "c128" in kn) else kn
        tuned = {"config": dict(tune.DEFAULT, **kn), "timings": None}
    elif getattr(args, "no_tune", False):
        tuned = {"config": dict(tune.DEFAULT), "timings": None}
    else:
        tuned = tune.tune_batch(insts, Ks, Bs, d3m.C64_IR, reps=1)
    cfg = tuned["config"]
    _log(f"tuned tile {tuned}")
    fs, Xs, flops = [], [], 0.0
    for inst, B in zip(insts, Bs):
        plan = d3m.Plan(inst.sizes, inst.pairs, grid=inst.grid, **cfg)
        flops += plan.info["flops_factor"]
        fs.append(d3m.Factor(plan, d3m.C64_IR, nrhs_max=16))
        Xs.append(torch.zeros_like(B))
    b = d3m.Batch(fs)
    b.run(Ks, Bs, Xs)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        b.run(Ks, Bs, Xs)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b.run(Ks, Bs, Xs)
    g.replay()
    torch.cuda.synchronize()
    e0, e1 = _events()
    e0.record()
    for _ in range(args.steps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    sts = [f.status() for f in fs]
    etas = [st["eta"] for st in sts]
    iters = [st["ir_iters"] for st in sts]
    ok = all(st["status"] == 0 for st in sts)
    # the same instances one after another (each its own launches), for comparison
    e0, e1 = _events()
    e0.record()
    for f, K, B, X in zip(fs, Ks, Bs, Xs):
        f.factorize(K)
        f.solve(B, X)
    e1.record()
    torch.cuda.synchronize()
    seq = e0.elapsed_time(e1)
    return {"metric": "batched frequency sweep: aggregate factor TFLOP/s and time for all instances",
            "value": flops / ms / 1e9, "unit": "TFLOP/s", "ms_per_sweep": ms, "sequential_ms": seq,
            "n_instances": len(insts), "status_ok": ok, "max_eta": max(etas), "ir_iters": sorted(set(iters)),
            "tuned": cfg, "tuner_ms": tuned["timings"], "factor_gflop_total": flops / 1e9, "dtype": "c64+c128",
            "data": "synthetic", "n_gpus": 1,
            "config": {"workload": "batch: 32-instance sweep, grids {2x2x2,3x3x2,4x4x2}, n~U{100..500}, "
                                   "f_k = 0.5 + 1.5k/31, 16 RHS each, hipGraph replay"}}


def diff(args):
    import torch

    import paper_2002_05026_amd as d3m
    from paper_2002_05026_amd import instances as gen
    t0 = time.perf_counter()
    inst = gen.config_diff(nrhs=128)
    _log(f"diff: N={inst.N}, K {inst.K.nbytes / 1e9:.1f} GB generated in {time.perf_counter() - t0:.0f}s")
    plan = d3m.Plan(inst.sizes, inst.pairs, grid=inst.grid)
    flops = plan.info["flops_factor"]
    _log(f"plan: {plan.info['ntask_factor']} factor tasks, {flops / 1e12:.1f} TFLOP")
    K = torch.from_numpy(inst.K).cuda()
    B = torch.from_numpy(inst.B).cuda()
    C = torch.from_numpy(inst.C).cuda()
    del inst.K
    X = torch.empty_like(B)
    f = d3m.Factor(plan, d3m.C64_IR, nrhs_max=128, timing=True)
    f.factorize(K)
    f.solve(B, X)
    torch.cuda.synchronize()
    st0 = f.status()
    _log(f"warm run status {st0['status']} eta {st0['eta_hist']}")
    e0, e1 = _events()
    e2, e3 = _events()
    e0.record()
    f.factorize(K)
    f.solve(B, X)
    e1.record()
    e2.record()
    Lam, dK = f.adjoint(X, C)
    e3.record()
    torch.cuda.synchronize()
    st = f.status()
    ms = e0.elapsed_time(e1)
    adj = e2.elapsed_time(e3)
    dag = st["t_factor_dag_ms"] / max(1, st["n_factor_dag"])
    J = float(torch.real((C * X).sum()))
    Jl = float(torch.real((Lam * B).sum()))
    return {"metric": "differentiation at scale: c64+IR time-to-solve, adjoint time, factor TFLOP/s",
            "value": flops / dag / 1e9, "unit": "TFLOP/s", "N": plan.N, "nrhs": 128,
            "time_to_solve_ms": ms, "adjoint_ms": adj, "factor_dag_ms": dag,
            "frac_fp32_peak": flops / dag / 1e9 / PEAK_FP32_MFMA, "status": st["status"],
            "eta_hist": st["eta_hist"], "J": J, "identity_rel_err": abs(J - Jl) / abs(J),
            "factor_gflop": flops / 1e9, "dtype": "c64+c128", "data": "synthetic", "n_gpus": 1,
            "config": {"workload": "diff: 6x6x6 domain grid, 540 interfaces, n~U{300..700}, 128 RHS, "
                                   "complex64 factor + FP64 refinement + adjoint"}}


def pivot(args):
    """The precision workload's K factored with and without in-tile pivoting."""
    import torch

    import paper_2002_05026_amd as d3m
    from paper_2002_05026_amd import instances as gen
    inst = gen.config_precision(nrhs=64)
    plan = d3m.Plan(inst.sizes, inst.pairs, grid=inst.grid)
    flops = plan.info["flops_factor"]
    K = torch.from_numpy(inst.K).cuda()
    B = torch.from_numpy(inst.B).cuda()
    X = torch.empty_like(B)
    out = {}
    for prec in (d3m.C64_IR, d3m.C128):
        for piv in (False, True):
            f = d3m.Factor(plan, prec, nrhs_max=64, timing=True, pivot=piv)
            f.factorize(K)
            f.solve(B, X)
            torch.cuda.synchronize()
            f.status()
            e0, e1 = _events()
            e0.record()
            for _ in range(args.steps):
                f.factorize(K)
                f.solve(B, X)
            e1.record()
            torch.cuda.synchronize()
            st = f.status()
            key = ("c64+IR" if prec == d3m.C64_IR else "c128") + (" pivoted" if piv else "")
            dag = st["t_factor_dag_ms"] / max(1, st["n_factor_dag"])
            out[key] = {"time_to_solve_ms": e0.elapsed_time(e1) / args.steps, "factor_dag_ms": dag,
                        "factor_tflops": flops / dag / 1e9, "eta": st["eta"], "ir_iters": st["ir_iters"],
                        "status": st["status"]}
            _log(f"pivot {key}: {out[key]}")
            del f
            torch.cuda.empty_cache()
    return {"metric": "in-tile Bunch-Kaufman pivoting: factor and time-to-solve against the unpivoted factor",
            "unit": "ms", "value": out["c64+IR pivoted"]["time_to_solve_ms"], "runs": out, "n_gpus": 1,
            "dtype": "c64+c128", "data": "synthetic",
            "config": {"workload": "pivot: the precision workload (4x4x4, N=%d, 64 RHS)" % inst.N}}


def primal(args):
    """Primal reduction -> reduced mixed solve -> primal recovery with ports."""
    import torch

    import paper_2002_05026_amd as d3m
    from paper_2002_05026_amd import instances as gen
    inst = gen.config_primal(nrhs=16)
    red = d3m.Plan(inst.sizes[:inst.nb], inst.pairs[:inst.npair_red], grid=inst.grid)
    order = [inst.nb + d for d in range(inst.ndom)] + red.order().tolist()
    plan = d3m.Plan(inst.sizes, inst.pairs, order=order, nelim=inst.ndom)
    _log(f"primal: N={inst.N} ({inst.ndom} interiors, reduced N={red.N}), "
         f"{plan.info['flops_factor'] / 1e9:.0f} GFLOP reduction, {red.info['flops_factor'] / 1e9:.0f} GFLOP dual")
    A = torch.from_numpy(inst.K).cuda()
    F = torch.from_numpy(inst.F).cuda()
    M = torch.from_numpy(inst.M).cuda()
    fp = d3m.Factor(plan, d3m.C128, nrhs_max=16, timing=True)
    fd = d3m.Factor(red, d3m.C64_IR, nrhs_max=16, timing=True)

    def step():
        Kred, G = fp.reduce(A, F)
        fd.factorize(Kred)
        Xred = fd.solve(G)
        return fp.recover(Xred, M)

    step()
    torch.cuda.synchronize()
    fp.status()
    fd.status()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    tr = td = tc = 0.0
    for _ in range(args.steps):
        ev[0].record()
        Kred, G = fp.reduce(A, F)
        ev[1].record()
        fd.factorize(Kred)
        Xred = fd.solve(G)
        ev[2].record()
        U, S = fp.recover(Xred, M)
        ev[3].record()
        torch.cuda.synchronize()
        tr += ev[0].elapsed_time(ev[1])
        td += ev[1].elapsed_time(ev[2])
        tc += ev[2].elapsed_time(ev[3])
    sp, sd = fp.status(), fd.status()
    n = args.steps
    return {"metric": "primal reduction + dual solve + primal recovery time", "unit": "ms",
            "value": (tr + td + tc) / n, "reduce_ms": tr / n, "dual_ms": td / n, "recover_ms": tc / n,
            "reduce_tflops": plan.info["flops_factor"] / (tr / n) / 1e9,
            "dual_eta": sd["eta"], "status": [sp["status"], sd["status"]], "N": inst.N, "N_reduced": red.N,
            "n_gpus": 1, "dtype": "c128 reduction + c64/c128 dual", "data": "synthetic",
            "config": {"workload": "primal: 4x4x4 domains, interfaces and interiors n~U{300..600}, 16 RHS, 8 ports"}}
