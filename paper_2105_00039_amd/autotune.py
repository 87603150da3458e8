"""Autotuner of the forward gather's launch shape.

The force gather keeps each lane's contacts in a list in LDS and drains it
into the Eq. 1 work before it can overflow.  Three knobs shape the launch:

* the list length (24 or 40 entries): a longer list drains less often, which
  pays when agents have many contacts (dense or clustered populations,
  FP64); a shorter one leaves LDS for more resident blocks;
* the block size (256 or 64 threads): the list's LDS and the wavefronts
  come in smaller units (one wavefront per block at 64), so blocks finish
  and are replaced one wavefront at a time and the batched step's
  per-block simulation lookup covers fewer agents;
* the run walk ("lanes" or "planes"): each lane takes all of its agent's 9
  stencil runs in turn (a wavefront then steps as often as its busiest lane
  has candidates), or the lanes take the z-planes together (their loads stay
  within one plane of slots, which pays on dense clustered populations).

Results are identical bit for bit for every choice (each agent's contacts
are summed in the same order by one lane), so the choice is decided by
timing the step on the caller's own workload, once per cache key.

The default key is (dtype, agent count to the nearest power of two, mean box
occupancy to the nearest half power of two, number of simulations).  Mean
occupancy counts empty boxes, so a clustered population looks sparse by it;
such callers pass their own ``key``.

``tune_box_order`` times the row order of a single simulation's boxes (row-
major or 16 x 16 tiles, the workspace's ``box_order``) the same way, over
grid build + step, since the order changes both; forces and displacements do
not depend on it either.
"""
from __future__ import annotations

import json
import math
import os

import torch

from . import MechStepError, device_status, grid_info

# (contact-list length, threads per block, run walk); the first is the
# library default
CHOICES = tuple((lst, nt, walk) for walk in ("lanes", "planes") for nt in (64, 256)
                for lst in (24, 40))


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


def _as_choice(v):
    """A cached entry as a (list, block, walk) triple (older caches hold the
    list only, or the list and block)."""
    if isinstance(v, (list, tuple)):
        return (int(v[0]), int(v[1]), str(v[2]) if len(v) > 2 else "lanes")
    return (int(v), 64, "lanes")


def _set(ws, c):
    ws.gather_list, ws.gather_block, ws.gather_walk = c


def tune(ws, step, key: str | None = None, choices=CHOICES, reps: int = 3, cache=None,
         margin: float = 0.02) -> dict:
    """Pick the fastest (list length, block size, run walk) for ``step`` (a callable
    running one force step on the workspace's current build, e.g. ``lambda:
    mech_step(ws, params, out=out)``) and set it on ``ws``.  The first of
    ``choices`` (the library default) is kept unless another is faster by more
    than ``margin``, so a tie does not flip the choice from run to run.

    cache: None, a dict, or the path of a JSON file (read if present, written
    after a timed choice).  Returns {"key", "choice": (list, block, walk),
    "source": "cache" | "timed", "ms": {"list/block/walk": mean ms per step}}."""
    choices = tuple(_as_choice(c) for c in choices)
    key = key or default_key(ws)
    table, path = _load(cache)
    if key in table and _as_choice(table[key]) in choices:
        c = _as_choice(table[key])
        _set(ws, c)
        return dict(key=key, choice=c, source="cache", ms={})
    times = {}
    for c in choices:
        _set(ws, c)
        times[c] = _time(step, reps)
    best = min(times, key=times.get)
    if times[choices[0]] <= times[best] * (1.0 + margin):
        best = choices[0]
    _set(ws, best)
    table[key] = list(best)
    if path is not None:
        with open(path, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
    return dict(key=key, choice=best, source="timed",
                ms={f"{c[0]}/{c[1]}/{c[2]}": t for c, t in times.items()})


def _time(fn, reps):
    fn()                                         # warm-up of this variant
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def tune_box_order(ws, build_and_step, key: str | None = None, reps: int = 5, cache=None,
                   margin: float = 0.03) -> dict:
    """Pick the faster row order ("rows" or "tiles") of a single simulation's
    boxes for ``build_and_step`` (a callable running one grid build and one
    step on the workspace, e.g. ``lambda: (grid_build(ws, x, y, z, d),
    mech_step(ws, params, out=out))``) and set it as ``ws.box_order``.  The
    order the automatic rule picks for this workload is kept unless the other
    is faster by more than ``margin``.  The last call leaves a build in the
    chosen order.  cache: as for :func:`tune` (entries "rows" / "tiles").
    An order whose build fails (tiles whose padded box count exceeds the
    workspace's max_boxes) is not chosen.
    Returns {"key", "choice", "auto", "source", "ms": {order: ms per call}}."""
    if ws.c.max_sims != 1:
        raise ValueError("tune_box_order: batched builds always number rows row-major")
    ws.box_order = "auto"
    build_and_step()
    auto = "tiles" if grid_info(ws)[0]["tile_shift"] else "rows"
    key = (key or default_key(ws)) + "|order"
    table, path = _load(cache)
    if table.get(key) in ("rows", "tiles"):
        ws.box_order = table[key]
        build_and_step()
        return dict(key=key, choice=table[key], auto=auto, source="cache", ms={})
    other = "tiles" if auto == "rows" else "rows"
    times = {}
    for c in (auto, other):
        ws.box_order = c
        try:
            build_and_step()
            device_status(ws)
        except MechStepError:
            continue
        times[c] = _time(build_and_step, reps)
    best = other if other in times and times[other] * (1.0 + margin) < times[auto] else auto
    ws.box_order = best
    build_and_step()
    table[key] = best
    if path is not None:
        with open(path, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
    return dict(key=key, choice=best, auto=auto, source="timed", ms=times)

