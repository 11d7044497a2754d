"""Benchmark of the D3M dual factorization and solution on one MI355X.

Workload (the precision configuration): a 4x4x4 domain grid, 144 interfaces
with n ~ U{300..600} unknowns (about 65k unknowns), synthetic seeded values
per the recipe in paper_2002_05026_amd/instances.py, 64 right-hand sides.
One step is the whole hot path on inputs already resident in HBM:
scatter/convert K, complex64 block LDL^T (one persistent DAG launch), block
solve, then FP64 residuals and refinement until eta_inf <= 1e-10, including
the certifying residual.  The FP64 path (complex128 factor + solve + one
certifying residual) is timed on the same K for the mixed-vs-FP64 speedup.

Prints one JSON line (see the design doc for every field).
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
TRAFFIC_BYTES = 222.45e9
TRAFFIC_SRC_HASH = "59fbe565b847a49b"
KERNEL_SOURCES = tuple("paper_2002_05026_amd/csrc/" + f for f in (
    "dag_kernels.hip", "gemm_engine.h", "tile_ldlt.h", "d3m_internal.h", "planner.cpp"))


def measured_traffic():
    import hashlib
    h = hashlib.sha1(b"".join(open(os.path.join(ROOT, p), "rb").read() for p in KERNEL_SOURCES)).hexdigest()[:16]
    return TRAFFIC_BYTES if h == TRAFFIC_SRC_HASH else None


def cpu_baseline(inst):
    """The CPU oracle (as it stands) on a bounded sample of the same workload:
    the principal submatrix of K on the interfaces inside the domain box
    [0,2)x[0,4)x[0,4) (a 2x4x4 half of the grid), factor + one 64-RHS solve."""
    import oracle
    from paper_2002_05026_amd import instances as gen
    keep = gen.box_interfaces(inst, (0, 0, 0), (2, 4, 4))
    sub = gen.subinstance(inst, keep)
    order = oracle.nd_order((2, 4, 4))
    p = oracle.OraclePlan(sub.sizes, sub.pairs, order)
    flops = p.stats()["flops"]
    t0 = time.perf_counter()
    p.factor(sub.K)
    t1 = time.perf_counter()
    p.solve(sub.B)
    t2 = time.perf_counter()
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": flops / (t1 - t0) / 1e12, "unit": "TFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"factor of the 2x4x4 half-grid principal submatrix ({len(keep)} interfaces, "
                      f"N={sub.N}, {flops / 1e9:.1f} GFLOP) in {t1 - t0:.2f} s; 64-RHS solve {t2 - t1:.2f} s",
            "factor_s": t1 - t0}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison path")
    ap.add_argument("--nrhs", type=int, default=64)
    ap.add_argument("--workload", default="precision", choices=["precision", "fp64", "batch", "diff"],
                    help="precision (default): the metric's workload; the others measure the remaining "
                         "configurations and print their own JSON line")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one plain 1 GiB device copy (for scaling HBM byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU path is a design "
              "(see DESIGN.md) and is not built.", file=sys.stderr)
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
        print(json.dumps(out), flush=True)
        return
    import paper_2002_05026_amd as d3m
    from paper_2002_05026_amd import instances as gen

    t0 = time.perf_counter()
    inst = gen.config_precision(nrhs=args.nrhs)
    print(f"[bench] instance N={inst.N} generated in {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    plan = d3m.Plan(inst.sizes, inst.pairs, grid=inst.grid)
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
    del f32
    torch.cuda.empty_cache()

    fp64 = None
    if not args.no_fp64:
        f64 = d3m.Factor(plan, d3m.C128, nrhs_max=args.nrhs, timing=True)
        ms64, st64 = timed(f64, max(2, args.steps // 2), 1)
        dag64 = st64["t_factor_dag_ms"] / max(1, st64["n_factor_dag"])
        fp64 = {"time_to_solve_ms": ms64, "factor_dag_ms": dag64, "factor_tflops": flops / dag64 / 1e9,
                "frac_fp64_peak": flops / dag64 / 1e9 / PEAK_FP64_MFMA, "eta": st64["eta"]}
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
                  "factor_dag_ms": dag_ms, "factor_tflops": achieved},
        "fp64": fp64,
        "roofline": {"kernel": "k_dag<float> (complex64 factor DAG)", "bound": "mfma", "achieved": achieved,
                     "peak": PEAK_FP32_MFMA, "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_MFMA,
                     "traffic": measured_traffic()},
        "cpu_baseline": {k: v for k, v in cpu.items() if k != "factor_s"} if cpu else None,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
