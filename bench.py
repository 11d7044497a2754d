"""Benchmark of the D3M dual factorization and solution on one MI355X.

Workload (the precision configuration): a 4x4x4 domain grid, 144 interfaces
with n ~ U{300..600} unknowns (about 65k unknowns), synthetic seeded values
per the recipe in paper_2002_05026_amd/instances.py, 64 right-hand sides.
One step is the whole hot path on inputs already resident in HBM:
scatter/convert K, complex64 block LDL^T (one persistent DAG launch), block
solve, then FP64 residuals and refinement until eta_inf <= 1e-10, including
the certifying residual.  The FP64 path (complex128 factor + solve + one
certifying residual) is timed on the same K for the mixed-vs-FP64 speedup.

Prints one JSON line: the metric, the whole-step rate, the roofline of the
factor DAG, the oracle's CPU baseline and the per-phase timings.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "block-LDLᵀ TFLOP/s + time-to-solve at 1e-10 residual, mixed+IR vs FP64"
PEAK_FP32_MFMA = 157.3   # TFLOP/s, MI355X dense FP32 matrix
PEAK_FP64_MFMA = 78.6    # TFLOP/s, MI355X dense FP64 matrix
# HBM bytes per complex64 factor-DAG launch on this workload, from the two
# rocprofv3 --pmc runs (FETCH_SIZE x2.0, WRITE_SIZE x1.0 after the plain-copy
# calibration) recorded in profiles/k_dag_factor_c64_precision_4x4x4.md, valid
# only for the kernel and planner sources they were taken with.
TRAFFIC_BYTES = 224.17e9
TRAFFIC_SRC_HASH = "40f35fbe27a62e7d"
KERNEL_SOURCES = tuple("paper_2002_05026_amd/csrc/" + f for f in (
    "dag_kernels.hip", "gemm_engine.h", "tile_ldlt.h", "tile_bk.h", "solve_mv.h", "launch.h", "d3m_internal.h",
    "planner.cpp"))


def measured_traffic():
    import hashlib
    h = hashlib.sha1(b"".join(open(os.path.join(ROOT, p), "rb").read() for p in KERNEL_SOURCES)).hexdigest()[:16]
    return TRAFFIC_BYTES if h == TRAFFIC_SRC_HASH else None


def host_cpu():
    """CPU model, logical CPUs and the CPUs this process may run on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count() or 1
    return {"cpu_model": model, "nproc": os.cpu_count() or 1, "usable_cpus": usable}


def oracle_threads():
    return int(os.environ.get("OMP_NUM_THREADS", host_cpu()["usable_cpus"]))


def oracle_factor_solve(inst, grid, keep=None):
    """Factor (and solve the instance's right-hand sides with) the CPU oracle
    as it stands; keep: the principal submatrix on these interfaces."""
    import oracle
    from paper_2002_05026_amd import instances as gen
    sub = gen.subinstance(inst, keep) if keep is not None else inst
    p = oracle.OraclePlan(sub.sizes, sub.pairs, oracle.nd_order(grid))
    flops = p.stats()["flops"]
    t0 = time.perf_counter()
    assert p.factor(sub.K) == -1
    t1 = time.perf_counter()
    p.solve(sub.B)
    t2 = time.perf_counter()
    return {"N": sub.N, "nblk": sub.nb, "gflop": flops / 1e9, "factor_s": t1 - t0, "solve_s": t2 - t1,
            "factor_tflops": flops / (t1 - t0) / 1e12}


def one_thread_sample():
    """Child process (OMP_NUM_THREADS=1): the oracle on the 2x2x2 corner box
    of the benchmark's workload; prints one JSON line."""
    from paper_2002_05026_amd import instances as gen
    inst = gen.config_precision(nrhs=64)
    keep = gen.box_interfaces(inst, (0, 0, 0), (2, 2, 2))
    r = oracle_factor_solve(inst, (2, 2, 2), keep)
    r["threads"] = oracle_threads()
    print(json.dumps(r), flush=True)


def cpu_baseline(inst):
    """The CPU oracle (as it stands, never tuned) on the benchmark's own
    workload with every host thread -- factor of the whole 4x4x4 matrix and
    the 64-RHS solve -- plus a 1-thread run on its 2x2x2 corner box."""
    import subprocess
    full = oracle_factor_solve(inst, inst.grid)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    one = None
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-one-thread"], env=env,
                       capture_output=True, text=True, timeout=600)
    if r.returncode == 0 and r.stdout.strip():
        one = json.loads(r.stdout.strip().splitlines()[-1])
    out = {"value": full["factor_tflops"], "unit": "TFLOP/s", "cores": oracle_threads(), "kind": "oracle",
           "sample": f"the whole workload: factor of K (N={full['N']}, {full['gflop']:.1f} GFLOP) in "
                     f"{full['factor_s']:.2f} s, then the 64-RHS solve in {full['solve_s']:.2f} s",
           "time_to_solve_s": full["factor_s"] + full["solve_s"]}
    out.update(host_cpu())
    if one:
        out["one_thread"] = {"sample": f"2x2x2 corner box ({one['nblk']} interfaces, N={one['N']}, "
                                       f"{one['gflop']:.1f} GFLOP), factor + 64-RHS solve",
                             "factor_tflops": one["factor_tflops"], "factor_s": one["factor_s"],
                             "solve_s": one["solve_s"], "threads": one["threads"]}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison path")
    ap.add_argument("--nrhs", type=int, default=64)
    ap.add_argument("--no-tune", action="store_true", help="default plan knobs instead of the autotuner's")
    ap.add_argument("--fp64-nrhs", default="1,16", help="right-hand-side counts of the fp64 workload")
    ap.add_argument("--knobs", default=None,
                    help='fixed plan knobs instead of the autotuner, JSON for both precisions or '
                         '{"c64": {...}, "c128": {...}} (e.g. to profile a tuned configuration)')
    ap.add_argument("--workload", default="precision", choices=["precision", "fp64", "batch", "diff", "pivot", "primal"],
                    help="precision (default): the metric's workload; the others measure the remaining "
                         "configurations and print their own JSON line")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one plain 1 GiB device copy (for scaling HBM byte counters) and exit")
    ap.add_argument("--cpu-one-thread", action="store_true", help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_one_thread:
        one_thread_sample()
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); a sharded multi-GPU path is "
              "not built.", file=sys.stderr)
        sys.exit(2)
    import torch
    if args.copy_calibration:
        x = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        y = torch.empty_like(x)
        x.fill_(1)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 1 << 30}))
        return
    if args.workload != "precision":
        from paper_2002_05026_amd import extra_workloads
        out = getattr(extra_workloads, args.workload)(args)
        if args.workload == "fp64" and not args.no_cpu:
            # the CPU oracle on the same 8x8x1 matrix: factor, then 1 and 16 RHS
            from paper_2002_05026_amd import instances as gen
            inst = gen.config_fp64(nrhs=16)
            r16 = oracle_factor_solve(inst, inst.grid)
            inst.B = inst.B[:1]
            r1 = oracle_factor_solve(inst, inst.grid)
            out["cpu_baseline"] = dict({"value": r16["factor_tflops"], "unit": "TFLOP/s", "kind": "oracle",
                                        "cores": oracle_threads(),
                                        "sample": "the whole 8x8x1 workload: factor, then 1 and 16 RHS",
                                        "factor_s": r16["factor_s"], "solve_1rhs_s": r1["solve_s"],
                                        "solve_16rhs_s": r16["solve_s"]}, **host_cpu())
        print(json.dumps(out), flush=True)
        return
    import paper_2002_05026_amd as d3m
    from paper_2002_05026_amd import instances as gen

    t0 = time.perf_counter()
    inst = gen.config_precision(nrhs=args.nrhs)
    print(f"[bench] instance N={inst.N} generated in {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    from paper_2002_05026_amd import tune
    tuned = {}
    for prec in ((d3m.C64_IR,) if args.no_fp64 else (d3m.C64_IR, d3m.C128)):
        if args.knobs:
            kn = json.loads(args.knobs)
            kn = kn.get("c64" if prec == d3m.C64_IR else "c128", kn) if ("c64" in kn or "c128" in kn) else kn
            tuned[prec] = {"config": dict(tune.DEFAULT, **kn), "timings": None}
        elif args.no_tune:
            tuned[prec] = {"config": dict(tune.DEFAULT), "timings": None}
        else:
            t0 = time.perf_counter()
            tuned[prec] = tune.tune(inst, prec, nrhs=args.nrhs, reps=2, save=False)
            print(f"[bench] tuned precision {prec} in {time.perf_counter() - t0:.0f}s: {tuned[prec]}",
                  file=sys.stderr, flush=True)
    plan = d3m.Plan(inst.sizes, inst.pairs, grid=inst.grid, **tuned[d3m.C64_IR]["config"])
    flops = plan.info["flops_factor"]
    K = torch.from_numpy(inst.K).cuda()
    B = torch.from_numpy(inst.B).cuda()
    X = torch.empty_like(B)
    torch.cuda.synchronize()

    def run(fac):
        fac.factorize(K)
        fac.solve(B, X)

    def timed(fac, steps, warmup):
        for _ in range(warmup):
            run(fac)
        torch.cuda.synchronize()
        fac.status()  # drain the event ring of the warmup steps
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(steps):
            run(fac)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        return ms, fac.status()

    f32 = d3m.Factor(plan, d3m.C64_IR, nrhs_max=args.nrhs, tol=1e-10, max_iter=10, timing=True)
    ms_mixed, st_mixed = timed(f32, args.steps, args.warmup)
    print(f"[bench] mixed: {ms_mixed:.2f} ms/step, status {st_mixed}", file=sys.stderr, flush=True)
    if st_mixed["status"] != 0:
        raise SystemExit(f"mixed path status {st_mixed}")
    dag_ms = st_mixed["t_factor_dag_ms"] / max(1, st_mixed["n_factor_dag"])
    # the first solve launch of each step is timed (the refinement's
    # launches run under the device stop flag and are not)
    solve_ms = st_mixed["t_solve_dag_ms"] / max(1, st_mixed["n_solve_dag"])
    solve_bytes = 2.0 * plan.info["nnz_L"] * 8
    del f32
    torch.cuda.empty_cache()

    fp64 = None
    if not args.no_fp64:
        plan64 = d3m.Plan(inst.sizes, inst.pairs, grid=inst.grid, **tuned[d3m.C128]["config"])
        f64 = d3m.Factor(plan64, d3m.C128, nrhs_max=args.nrhs, timing=True)
        ms64, st64 = timed(f64, max(2, args.steps // 2), 1)
        dag64 = st64["t_factor_dag_ms"] / max(1, st64["n_factor_dag"])
        s64 = st64["t_solve_dag_ms"] / max(1, st64["n_solve_dag"])
        fp64 = {"time_to_solve_ms": ms64, "factor_dag_ms": dag64, "factor_tflops": flops / dag64 / 1e9,
                "frac_fp64_peak": flops / dag64 / 1e9 / PEAK_FP64_MFMA, "eta": st64["eta"],
                "solve_dag_ms": s64, "solve_GBps": 2.0 * plan64.info["nnz_L"] * 16 / s64 / 1e6,
                "tuned": tuned[d3m.C128]["config"]}
        print(f"[bench] fp64: {ms64:.2f} ms/step, status {st64}", file=sys.stderr, flush=True)
        del f64
        torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(inst)
        print(f"[bench] cpu oracle: {cpu}", file=sys.stderr, flush=True)

    achieved = flops / dag_ms / 1e9
    out = {
        "metric": METRIC,
        "value": flops / ms_mixed / 1e9,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_mixed,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64+c128",
        "data": "synthetic",
        "config": {"workload": "precision: 4x4x4 domain grid, 144 interfaces, n~U{300..600} (N=%d), %d RHS, "
                               "complex64 factor + FP64 refinement to eta_inf<=1e-10" % (inst.N, args.nrhs),
                   "N": inst.N, "nrhs": args.nrhs, "factor_gflop": flops / 1e9,
                   "parallelism": "single GPU, persistent DAG"},
        "time_to_solve_ms": {"mixed_ir": ms_mixed, "fp64": fp64["time_to_solve_ms"] if fp64 else None},
        "speedup_mixed_vs_fp64": (fp64["time_to_solve_ms"] / ms_mixed) if fp64 else None,
        "mixed": {"eta": st_mixed["eta"], "eta_hist": st_mixed["eta_hist"], "ir_iters": st_mixed["ir_iters"],
                  "factor_dag_ms": dag_ms, "factor_tflops": achieved, "solve_dag_ms": solve_ms,
                  "solve_GBps": solve_bytes / solve_ms / 1e6,
                  "solve_tflops": plan.info["solve_flops_per_rhs"] * args.nrhs / solve_ms / 1e9},
        "tuned": {"config": tuned[d3m.C64_IR]["config"], "timings_ms": tuned[d3m.C64_IR]["timings"]},
        "fp64": fp64,
        "roofline": {"kernel": "k_dag<float> (complex64 factor DAG)", "bound": "mfma", "achieved": achieved,
                     "peak": PEAK_FP32_MFMA, "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_MFMA,
                     "traffic": measured_traffic()},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
