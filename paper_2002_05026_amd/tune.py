"""Tile-size tuner.

The planner splits every interface into tiles of at most `tile` rows; the
tile edge sets the grain of the factor DAG (bigger tiles: fewer tasks and
more work per MFMA tile product; smaller tiles: shorter critical path on
small fronts).  The paper weighs its dual tasks with benchmarked GEMM,
sytrf and triSolve timings (Sec. II); here the whole factor is timed on the
device for each candidate edge and the fastest is kept, per precision and
size bucket, in a JSON cache keyed by the GPU architecture.

Cache file: $D3M_TUNE_CACHE, else ~/.cache/d3m_tune.json.
"""
from __future__ import annotations

import json
import os
from typing import Optional, Sequence

CANDIDATES = (64, 96, 128)


def _cache_path() -> str:
    return os.environ.get("D3M_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "d3m_tune.json"))


def _arch() -> str:
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def size_bucket(mean_n: float) -> str:
    return "n<=256" if mean_n <= 256 else ("n<=512" if mean_n <= 512 else "n>512")


def load() -> dict:
    try:
        with open(_cache_path()) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def lookup(precision: int, mean_n: float, default: int = 128) -> int:
    try:
        key = f"{_arch()}/{precision}/{size_bucket(mean_n)}"
    except Exception:
        return default
    return int(load().get(key, {}).get("tile", default))


def tune(instance, precision: int, candidates: Sequence[int] = CANDIDATES, reps: int = 3,
         save: bool = True) -> dict:
    """Time the factorization of `instance` for each tile edge; return and
    cache {'tile': best, 'ms': {tile: ms}}."""
    import torch

    import paper_2002_05026_amd as d3m
    K = torch.from_numpy(instance.K).cuda()
    times = {}
    for tile in candidates:
        plan = d3m.Plan(instance.sizes, instance.pairs, grid=instance.grid, tile=tile)
        f = d3m.Factor(plan, precision, nrhs_max=1)
        f.factorize(K)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            f.factorize(K)
        e1.record()
        torch.cuda.synchronize()
        times[int(tile)] = e0.elapsed_time(e1) / reps
        st = f.status()
        if st["status"] not in (0,):
            raise RuntimeError(f"tuning factorization failed: {st}")
        del f
    best = min(times, key=times.get)
    res = {"tile": best, "ms": times}
    if save:
        mean_n = float(instance.sizes.mean())
        key = f"{_arch()}/{precision}/{size_bucket(mean_n)}"
        data = load()
        data[key] = res
        path = _cache_path()
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)
        os.replace(tmp, path)
    return res
