"""Tile-shape autotuner for the C-pass and W-update kernels (nmf_desc.tile_cfg).

A tile configuration is a pair (wc, cf): wc in {1, 2, 4} C-pass row groups per
64-column tile (1 = one wave per 16-column tile over the whole row chunk,
throughput; 2 / 4 = the chunk's rows split over the waves, shorter dependency
chains, latency), cf in {4, 16} W-update columns per tile.  Every
configuration computes the same iteration; the C-pass sum order depends on
wc, so configurations agree to rounding, and one plan gives the same bits
alone and in a batch.

The tuner times each candidate on the device for a workload -- one solve, or
one grouped batch of solves -- and keeps the fastest, optionally in a JSON
cache keyed by the workload's shape class, which `choose` reads back.
"""
from __future__ import annotations

import json
import os
import time
from typing import Dict, Iterable, List, Optional, Sequence, Tuple

import numpy as np

import paper_1009_0881_amd as P

CANDIDATES: List[Tuple[int, int]] = [(1, 16), (1, 4), (2, 16), (2, 4), (4, 16), (4, 4)]

_DESC_KEYS = ("m", "n", "r", "levels", "algo", "cycle", "prec")


def shape_key(plan_kwargs: dict, context: str = "solve") -> str:
    """Cache key of a workload: its shape class and the launch context."""
    parts = [context] + [f"{k}={plan_kwargs.get(k, '')}" for k in _DESC_KEYS]
    return ";".join(parts)


def _median_ms(samples: Sequence[float]) -> float:
    return float(np.median(np.asarray(samples))) * 1e3


def tune_solve(plan_kwargs: dict, M: np.ndarray, V0: np.ndarray, W0: np.ndarray, iters: int,
               candidates: Iterable[Tuple[int, int]] = CANDIDATES, repeats: int = 3) -> dict:
    """Time one solve of (M, V0, W0) under every candidate tile configuration.

    Returns {"best": (wc, cf), "tile_cfg": int, "ms": {"wc,cf": median ms}}.
    """
    import torch
    Md, V0d, W0d = P.to_device(M, V0, W0)
    timings: Dict[str, float] = {}
    best, best_ms = None, float("inf")
    for wc, cf in candidates:
        pl = P.Plan(**dict(plan_kwargs, tile_cfg=(wc, cf)))
        ws = pl.workspace()
        samples = []
        for rep in range(repeats + 1):
            V, W = V0d.clone(), W0d.clone()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            pl.solve(Md, V, W, iters, workspace=ws)
            torch.cuda.synchronize()
            if rep > 0:                      # first run: warm-up
                samples.append(time.perf_counter() - t0)
        ms = _median_ms(samples)
        timings[f"{wc},{cf}"] = ms
        if ms < best_ms:
            best, best_ms = (wc, cf), ms
    return {"best": best, "tile_cfg": P.tile(*best), "ms": timings}


def tune_batch(plan_kwargs: Sequence[dict], Ms, V0s, W0s, iters: Sequence[int],
               candidates: Iterable[Tuple[int, int]] = CANDIDATES, repeats: int = 2) -> dict:
    """Time one grouped batch (nmf_solve_batch) of the given problems under
    every candidate, all problems sharing the candidate's tiles."""
    import torch
    dev = [P.to_device(M, V0, W0) for M, V0, W0 in zip(Ms, V0s, W0s)]
    timings: Dict[str, float] = {}
    best, best_ms = None, float("inf")
    for wc, cf in candidates:
        plans = [P.Plan(**dict(kw, tile_cfg=(wc, cf))) for kw in plan_kwargs]
        samples = []
        for rep in range(repeats + 1):
            Vs = [d[1].clone() for d in dev]
            Ws = [d[2].clone() for d in dev]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            P.solve_batch(plans, [d[0] for d in dev], Vs, Ws, list(iters))
            torch.cuda.synchronize()
            if rep > 0:
                samples.append(time.perf_counter() - t0)
        ms = _median_ms(samples)
        timings[f"{wc},{cf}"] = ms
        if ms < best_ms:
            best, best_ms = (wc, cf), ms
    return {"best": best, "tile_cfg": P.tile(*best), "ms": timings}


def load_cache(path: str) -> dict:
    if not path or not os.path.exists(path):
        return {}
    with open(path) as fh:
        return json.load(fh)


def save_result(path: str, key: str, result: dict) -> None:
    cache = load_cache(path)
    cache[key] = {"best": list(result["best"]), "tile_cfg": result["tile_cfg"],
                  "ms": result["ms"]}
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def choose(plan_kwargs: dict, context: str = "solve", cache_path: Optional[str] = None) -> int:
    """tile_cfg for a workload: the cached tuning result, else 0 (the library's
    default tiles)."""
    entry = load_cache(cache_path).get(shape_key(plan_kwargs, context)) if cache_path else None
    if not entry:
        return 0
    wc, cf = entry["best"]
    return P.tile(wc, cf)
