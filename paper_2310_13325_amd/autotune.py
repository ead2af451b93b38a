"""Autotuner for the time-stepping kernel and the gradient's memory schedule,
with a JSON table.

The blocked kernel comes in a few tile shapes (extended tile size, rows per
thread, steps per launch); which one is fastest depends on the grid (how
evenly the interior tiles cover it), the number of pairs and the device.
`tune` times each candidate on the caller's own workload with HIP events on
the current stream, keeps the fastest, and records it in a `TileTable` keyed
by the grid and time length (or by the whole batch), saved as JSON so later
runs reuse the measurement.

`tune_schedule` does the same for how vip_grad_logpost spends device memory:
the number of final steps whose a^n the forward sweep keeps (each one saves
recomputing a step in the backward sweep) and the number of pairs simulated
at once (fewer live pairs leave room to keep more steps).
"""
from __future__ import annotations

import json
import os
from typing import Callable, Iterable, Optional

import torch

from . import binding as vb


def candidates(include_one_step: bool = True):
    c = list(range(vb.lib().vip_tile_count()))
    return ([-1] if include_one_step else []) + c


def key_for(grid: vb.Grid, npairs: int) -> str:
    return f"grid{grid.nx + 2 * grid.nb}x{grid.nz + 2 * grid.nb}:nt{grid.nt}:pairs{npairs}"


def key_for_batch(problems) -> str:
    return "batch:" + "|".join(key_for(p.grid, p.vel.shape[0] * p.geom.ns) for p in problems)


class TileTable:
    def __init__(self, path: Optional[str] = None):
        self.path = path
        self.entries = {}
        if path and os.path.exists(path):
            with open(path) as f:
                self.entries = json.load(f)

    def get(self, key: str) -> Optional[int]:
        e = self.entries.get(key)
        return None if e is None else int(e["tile"])

    def put(self, key: str, tile: int, timings_ms: dict, **extra):
        self.entries[key] = {"tile": int(tile), "ms": {str(k): v for k, v in timings_ms.items()},
                             "device": torch.cuda.get_device_name(0), **extra}
        if self.path:
            tmp = self.path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(self.entries, f, indent=1, sort_keys=True)
            os.replace(tmp, self.path)


def time_ms(fn: Callable[[], object], reps: int = 1) -> float:
    fn()                                   # warm: first use may capture or allocate
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(reps):
        fn()
    stop.record()
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / reps


def tune(ctx: vb.Context, fn: Callable[[], object], key: str, table: Optional[TileTable] = None,
         tiles: Optional[Iterable[int]] = None, reps: int = 1) -> int:
    """Use the tabulated tile for `key`, or time `fn` under each candidate
    tile, pick the fastest, record it; leaves the context set to it."""
    if table is not None:
        t = table.get(key)
        if t is not None:
            ctx.set_tile(t)
            return t
    timings = {}
    for t in (candidates() if tiles is None else tiles):
        ctx.set_tile(t)
        try:
            timings[t] = time_ms(fn, reps)
        except vb.VipError as e:
            if e.status != -7:                 # unsupported shape for this call: skip it
                raise
    best = min(timings, key=timings.get)
    ctx.set_tile(best)
    if table is not None:
        table.put(key, best, timings)
    return best


def schedules(grid: vb.Grid, geom: vb.Geometry, npart: int, ckpt_every: int,
              budget_bytes: int):
    """Candidate (stored_steps, live_pairs) for a workspace budget: recompute
    everything with all pairs live; all pairs live with the longest stored tail
    that fits; every step stored with the most live pairs that fit, and with
    the pairs split evenly over the same number of chunks."""
    pairs = npart * geom.ns
    m = grid.nt - 1
    size = lambda s, live: vb.grad_logpost_workspace_bytes(grid, geom, npart, ckpt_every, live, s)
    out = [(0, 0)]
    s_all = vb.stored_steps_for_budget(grid, geom, npart, ckpt_every, budget_bytes, 0)
    if s_all > 0:
        out.append((s_all, 0))
    if s_all < m:
        lo, hi = 0, pairs           # most live pairs that store every step
        while hi - lo > 1:
            mid = (lo + hi) // 2
            if size(m, mid) <= budget_bytes:
                lo = mid
            else:
                hi = mid
        if lo > 0:
            out.append((m, lo))
            chunks = -(-pairs // lo)
            even = -(-pairs // chunks)
            if even != lo:
                out.append((m, even))
    return [c for c in out if size(*c) <= budget_bytes]


def tune_schedule(fn: Callable[[int, int], object], key: str, cands,
                  table: Optional[TileTable] = None, reps: int = 1):
    """Use the tabulated (stored_steps, live_pairs) for `key`, or time
    fn(stored_steps, live_pairs) for each candidate and keep the fastest."""
    if table is not None:
        e = table.entries.get(key)
        if e is not None and "stored_steps" in e:
            return int(e["stored_steps"]), int(e["live_pairs"])
    timings = {}
    for s, live in cands:
        timings[(s, live)] = time_ms(lambda: fn(s, live), reps)
    best = min(timings, key=timings.get)
    if table is not None:
        table.put(key, -2, {f"{s}/{live}": t for (s, live), t in timings.items()},
                  stored_steps=best[0], live_pairs=best[1])
    return best


def tune_joint(ctx: vb.Context, fn: Callable[[int, int], object], cands,
               tiles: Optional[Iterable[int]] = None, reps: int = 1):
    """Time fn(stored_steps, live_pairs) for every tile shape and schedule in
    `cands` (the best tile depends on the schedule: keeping every step trades
    the recompute sweep for a store in the forward one) and keep the fastest.
    Leaves the context set to the chosen tile; returns (tile, stored, live, timings)."""
    timings = {}
    for t in (candidates(False) if tiles is None else tiles):
        ctx.set_tile(t)
        for st, live in cands:
            try:
                timings[(t, st, live)] = time_ms(lambda: fn(st, live), reps)
            except vb.VipError as e:
                if e.status != -7:
                    raise
    best = min(timings, key=timings.get)
    ctx.set_tile(best[0])
    return best[0], best[1], best[2], timings
