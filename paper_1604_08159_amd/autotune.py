"""Stencil tile autotuner.

For each (J, p, precision) asked for, every valid tile edge is timed on the
GPU: a small batch of resident two-vortex solves of that size is created with
the candidate tile, warmed up, and stepped through solve_batch (graph replay)
on a private stream; the edge with the lowest time per step wins.  The
choices go to the library's tile table (mra_tune_set_tile), so solves created
afterwards take them, and can be kept in a JSON cache keyed by device name:

    {"device": "...", "entries": {"J9_p2_prec2": {"tile": 32,
                                                  "ms_per_step": {"16": ..., "32": ...}}}}

Timing uses the same launches as the step (no separate micro-benchmark), so
the choice accounts for everything the tile changes: halo re-reads of the
residual, product and scalar stencils and the blocks per CU their LDS allows.
"""
from __future__ import annotations

import json
import math
import os
import time
from typing import Dict, Iterable, Optional, Tuple

import torch

from . import Solve, flow_desc, grid_desc, solve_batch, tune_get_tile, tune_set_tile, MRA_FP64

CANDIDATES = (8, 16, 32)


def valid_tiles(J: int, p: int, prec: int) -> Tuple[int, ...]:
    """The edges the library accepts for (J, p, prec)."""
    bulk64 = prec == MRA_FP64
    return tuple(t for t in CANDIDATES if t <= (1 << J) and not (bulk64 and p == 3 and t == 32))


def _pair_field(N: int, b: float, r0: float = 0.3) -> torch.Tensor:
    """Two Gaussian vortices (unit circulation, radius r0) at (pi -/+ b/2, pi)."""
    h = 2 * math.pi / N
    x = torch.arange(N, dtype=torch.float64) * h
    X, Y = x[None, :], x[:, None]
    w = torch.zeros((N, N), dtype=torch.float64)
    for cx in (math.pi - b / 2, math.pi + b / 2):
        w += torch.exp(-((X - cx) ** 2 + (Y - math.pi) ** 2) / r0 ** 2) / (math.pi * r0 ** 2)
    return w


def time_tile(J: int, p: int, prec: int, tile: int, nsolves: int = 4, steps: int = 8, warmup: int = 2,
              m: int = 20, eps: float = 1e-4, device: str = "cuda:0") -> float:
    """Milliseconds per step of a batch of nsolves two-vortex solves of
    (J, p, prec) laid out with the given tile edge."""
    dev = torch.device(device)
    prev = tune_get_tile(J, p, prec)
    tune_set_tile(J, p, prec, tile)
    st = torch.cuda.Stream(device=dev)
    solves = []
    try:
        with torch.cuda.stream(st):
            for i in range(nsolves):
                w0 = _pair_field(1 << J, 1.0 + 0.1 * i).to(dev)
                solves.append(Solve(grid_desc(J, p, eps), flow_desc(2e-4, 0.17), prec, m, 0.01, w0, stream=st))
        solve_batch(solves, [warmup] * nsolves, stream=st)
        st.synchronize()
        t0 = time.perf_counter()
        solve_batch(solves, [steps] * nsolves, stream=st)
        st.synchronize()
        return (time.perf_counter() - t0) / steps * 1e3
    finally:
        for s in solves:
            s.close()
        tune_set_tile(J, p, prec, prev if prev in valid_tiles(J, p, prec) else 0)


def entry_key(J: int, p: int, prec: int) -> str:
    return f"J{J}_p{p}_prec{prec}"


def parse_entry_key(k: str) -> Tuple[int, int, int]:
    j, p, prec = k.split("_")
    return int(j[1:]), int(p[1:]), int(prec[4:])


def autotune(configs: Iterable[Tuple[int, int, int]], cache: Optional[str] = None, device: str = "cuda:0",
             **timing) -> Dict[str, dict]:
    """Tunes every (J, p, prec) in configs that the cache does not already
    hold for this device, applies all choices, and rewrites the cache."""
    name = torch.cuda.get_device_name(torch.device(device))
    entries: Dict[str, dict] = {}
    if cache and os.path.exists(cache):
        with open(cache) as f:
            data = json.load(f)
        if data.get("device") == name:
            entries = dict(data.get("entries", {}))
    for J, p, prec in configs:
        k = entry_key(J, p, prec)
        if k not in entries:
            ms = {str(t): time_tile(J, p, prec, t, device=device, **timing) for t in valid_tiles(J, p, prec)}
            best = min(ms, key=ms.get)
            entries[k] = {"tile": int(best), "ms_per_step": ms}
        tune_set_tile(J, p, prec, entries[k]["tile"])
    if cache:
        tmp = cache + ".tmp"
        with open(tmp, "w") as f:
            json.dump({"device": name, "entries": entries}, f, indent=1)
        os.replace(tmp, cache)
    return entries


def apply_cache(cache: str, device: str = "cuda:0") -> int:
    """Applies a cache written for this device; returns the entries applied."""
    with open(cache) as f:
        data = json.load(f)
    if data.get("device") != torch.cuda.get_device_name(torch.device(device)):
        return 0
    n = 0
    for k, e in data.get("entries", {}).items():
        J, p, prec = parse_entry_key(k)
        tune_set_tile(J, p, prec, int(e["tile"]))
        n += 1
    return n
