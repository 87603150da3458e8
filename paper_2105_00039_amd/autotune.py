"""Autotuner of the forward gather's contact-list length.

The force gather keeps each lane's contacts in a list in LDS and drains it
into the Eq. 1 work before it can overflow.  A longer list drains less often,
which pays when agents have many contacts (dense or clustered populations,
FP64); a shorter one leaves LDS for more resident blocks, which pays at low
density.  Results are identical bit for bit for every length (the contacts
are summed in the same order), so the choice is decided by timing the step
on the caller's own workload, once per cache key.

The default key is (dtype, agent count to the nearest power of two, mean box
occupancy to the nearest half power of two, number of simulations).  Mean
occupancy counts empty boxes, so a clustered population looks sparse by it;
such callers pass their own ``key``.
"""
from __future__ import annotations

import json
import math
import os

import torch

from . import grid_info

CHOICES = (32, 40)


def default_key(ws) -> str:
    geo = grid_info(ws)
    n = max(ws.n_agents, 1)
    boxes = max(sum(g["n_boxes"] for g in geo), 1)
    return (f"{ws.dtype_name}|n2^{round(math.log2(n))}|occ2^{round(2 * math.log2(n / boxes)) / 2:g}"
            f"|sims{max(ws.n_sims, 1)}")


def _load(cache):
    if cache is None:
        return {}, None
    if isinstance(cache, dict):
        return cache, None
    path = os.fspath(cache)
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f), path
    return {}, path


def tune(ws, step, key: str | None = None, choices=CHOICES, reps: int = 3, cache=None,
         margin: float = 0.02) -> dict:
    """Pick the fastest contact-list length for ``step`` (a callable running one
    force step on the workspace's current build, e.g. ``lambda: mech_step(ws,
    params, out=out)``) and set it on ``ws``.  The first of ``choices`` (the
    library default) is kept unless another is faster by more than ``margin``,
    so a tie does not flip the choice from run to run.

    cache: None, a dict, or the path of a JSON file (read if present, written
    after a timed choice).  Returns {"key", "choice", "source": "cache" |
    "timed", "ms": {length: mean ms per step}}."""
    key = key or default_key(ws)
    table, path = _load(cache)
    if key in table and int(table[key]) in choices:
        ws.gather_list = int(table[key])
        return dict(key=key, choice=ws.gather_list, source="cache", ms={})
    times = {}
    for c in choices:
        ws.gather_list = c
        step()                                   # warm-up of this variant
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            step()
        b.record()
        torch.cuda.synchronize()
        times[c] = a.elapsed_time(b) / reps
    best = min(times, key=times.get)
    if times[choices[0]] <= times[best] * (1.0 + margin):
        best = choices[0]
    ws.gather_list = best
    table[key] = best
    if path is not None:
        with open(path, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
    return dict(key=key, choice=best, source="timed", ms=times)
