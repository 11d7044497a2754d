"""Autotuner of the plan's tile knobs.

The paper weighs its dual tasks with benchmarked GEMM, sytrf and triSolve
timings (Sec. II) to schedule them; here the knobs that set the grain of the
GPU task DAGs are chosen by timing the library itself on the device:

* tile        edge of the factor tiles (FACT/TRSM/update grain)      -> factor DAG time
* merge       source panels per merged Schur update task            -> factor DAG time
* solve_tile  rows of a solve task                                  -> solve DAG time
* rhs_groups  column groups of the right-hand sides (grouped DAG)   -> solve DAG time

A batch (tune_batch) is tuned as a batch: every knob by the time of the
whole merged run (factor, solve and refinement of all instances), since the
grain that is best for one instance alone (little parallelism) is not the
best for many merged into one launch.

Coordinate descent in that order: each knob's candidates are timed with the
best values found so far for the others, and a candidate replaces the
current value only when more than 0.5% faster (factor knobs by the time of
d3m_factorize, solve knobs by the time of d3m_solve for the caller's number
of right-hand sides, HIP events on the stream), and the fastest is kept.  Results are cached as JSON keyed
by GPU architecture, precision, interface-size bucket and right-hand-side
bucket.  Cache file: $D3M_TUNE_CACHE, else ~/.cache/d3m_tune.json.
"""
from __future__ import annotations

import json
import os
from typing import Optional

KNOBS = (("tile", (64, 96, 128)), ("merge", (4, 8, 12)), ("solve_tile", (32, 64, 128)), ("rhs_groups", (1, 2, 4)))
DEFAULT = {"tile": 128, "merge": 8, "solve_tile": 64, "rhs_groups": 1}
FACTOR_KNOBS = ("tile", "merge")


def _cache_path() -> str:
    return os.environ.get("D3M_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "d3m_tune.json"))


def _arch() -> str:
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def size_bucket(mean_n: float) -> str:
    return "n<=256" if mean_n <= 256 else ("n<=512" if mean_n <= 512 else "n>512")


def rhs_bucket(nrhs: int) -> str:
    return "1" if nrhs <= 1 else ("<=16" if nrhs <= 16 else ("<=64" if nrhs <= 64 else ">64"))


def key(precision: int, mean_n: float, nrhs: int) -> str:
    return f"{_arch()}/{precision}/{size_bucket(mean_n)}/rhs{rhs_bucket(nrhs)}"


def load() -> dict:
    try:
        with open(_cache_path()) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def lookup(precision: int, mean_n: float, nrhs: int) -> dict:
    """The cached configuration for this bucket, else the defaults."""
    try:
        k = key(precision, mean_n, nrhs)
    except Exception:
        return dict(DEFAULT)
    return dict(load().get(k, {}).get("config", DEFAULT))


def _time(instance, precision: int, nrhs: int, cfg: dict, reps: int) -> tuple:
    """(factorize ms, solve ms) of one configuration, means over reps (HIP
    events on the stream around the calls; what the knobs do not touch --
    scatter, norms, residuals -- is the same for every candidate)."""
    import numpy as np
    import torch

    import paper_2002_05026_amd as d3m
    plan = d3m.Plan(instance.sizes, instance.pairs, grid=instance.grid, **cfg)
    K = torch.from_numpy(instance.K).cuda()
    B = torch.from_numpy(np.ascontiguousarray(instance.B[:nrhs])).cuda()
    X = torch.empty_like(B)
    f = d3m.Factor(plan, precision, nrhs_max=nrhs)
    f.factorize(K)
    f.solve(B, X)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    tf = ts = 0.0
    for _ in range(reps):
        ev[0].record()
        f.factorize(K)
        ev[1].record()
        f.solve(B, X)
        ev[2].record()
        torch.cuda.synchronize()
        tf += ev[0].elapsed_time(ev[1])
        ts += ev[1].elapsed_time(ev[2])
    st = f.status()
    if st["status"] != 0:
        raise RuntimeError(f"tuning run failed: {st}")
    return tf / reps, ts / reps


# A candidate replaces the current value only when it is faster by more than
# this fraction: two timings closer than that are run-to-run noise, and a
# noise-level switch would make the chosen configuration change between runs.
MARGIN = 0.005


def _pick(times: dict, current: int) -> int:
    best = min(times, key=times.get)
    if current in times and times[best] >= (1.0 - MARGIN) * times[current]:
        return current
    return best


def tune(instance, precision: int, nrhs: Optional[int] = None, reps: int = 2, save: bool = True,
         knobs=KNOBS) -> dict:
    """Coordinate descent over the knobs on `instance`; returns (and caches)
    {'config': best, 'timings': {knob: {value: ms}}, 'key': cache key}."""
    if nrhs is None:
        nrhs = int(instance.B.shape[0])
    cfg = dict(DEFAULT)
    timings = {}
    for name, cands in knobs:
        times = {}
        for v in cands:
            trial = dict(cfg, **{name: v})
            fac, sol = _time(instance, precision, nrhs, trial, reps)
            times[int(v)] = fac if name in FACTOR_KNOBS else sol
        cfg[name] = _pick(times, cfg[name])
        timings[name] = times
    mean_n = float(instance.sizes.mean())
    res = {"config": cfg, "timings": timings, "key": key(precision, mean_n, nrhs)}
    if save:
        data = load()
        data[res["key"]] = res
        path = _cache_path()
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)
        os.replace(tmp, path)
    return res


def _time_batch(instances, Ks, Bs, precision: int, cfg: dict, reps: int) -> float:
    """ms of one d3m_batch_run (all instances, this configuration), mean over
    reps, after one untimed run."""
    import torch

    import paper_2002_05026_amd as d3m
    nrhs = int(Bs[0].shape[0])
    fs = [d3m.Factor(d3m.Plan(i.sizes, i.pairs, grid=i.grid, **cfg), precision, nrhs_max=nrhs) for i in instances]
    b = d3m.Batch(fs)
    Xs = [torch.empty_like(B) for B in Bs]
    b.run(Ks, Bs, Xs)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.run(Ks, Bs, Xs)
    e1.record()
    torch.cuda.synchronize()
    bad = [st for st in (f.status() for f in fs) if st["status"] != 0]
    if bad:
        raise RuntimeError(f"tuning run failed: {bad[0]}")
    del b, fs, Xs
    torch.cuda.empty_cache()
    return e0.elapsed_time(e1) / reps


def tune_batch(instances, Ks, Bs, precision: int, reps: int = 2, knobs=KNOBS) -> dict:
    """Coordinate descent over the knobs, each candidate timed as a whole
    batch run of `instances` (device K and B given); returns {'config': best,
    'timings': {knob: {value: ms}}} (not cached: a batch is its own case)."""
    cfg = dict(DEFAULT)
    timings = {}
    for name, cands in knobs:
        times = {}
        for v in cands:
            times[int(v)] = _time_batch(instances, Ks, Bs, precision, dict(cfg, **{name: v}), reps)
        cfg[name] = _pick(times, cfg[name])
        timings[name] = times
    return {"config": cfg, "timings": timings}
