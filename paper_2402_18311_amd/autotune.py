"""Timing-based choice of the charge scatter's grouping policy for a netlist and a batch of
slots (the tunable of the batched path; results never depend on it, only speed).

The scatter groups cells by bin tile and rebuilds the grouping every few evaluations; how
often, and whether the rebuilding evaluation accumulates in the old grouping (one launch
fewer) or the new one (no stale cells), depends on how far cells move per iteration, which
differs between netlists and between the early and late phases of a placement.  tune_scatter
times each candidate on scratch slots that start from the given slots' current positions (the
optimiser restarts there) and keeps the fastest.  A JSON cache keyed by the netlist's shape
and the batch size skips the timing.

    best = tune_scatter(pl, slots, gamma)            # applies and returns (every, deferred)
"""
from __future__ import annotations

import json
import os
import time

# (regroup_every, deferred); rebuilding at every evaluation pays off while cells still move by
# many bins per step (the first iterations from random positions, when they clump)
CANDIDATES = ((4, True), (4, False), (8, True), (2, True), (2, False), (1, False))


def _key(pl, k):
    nl = pl.nl
    return (f"cells{nl.n_cells}_pins{len(nl.pin_cell)}_bins{nl.mx}x{nl.my}"
            f"_p{pl.precision}_k{k}")


def tune_scatter(pl, slots, gamma, candidates=CANDIDATES, warm=8, iters=24, repeats=3,
                 cache=None):
    """Time `iters` iterations (after `warm`) of every (regroup_every, deferred) candidate on
    scratch slots holding the given slots' current positions; apply the fastest (median of
    `repeats`) to the placer's netlist and return it with the timings in ms per iteration."""
    import torch
    slots = [int(s) for s in (slots if isinstance(slots, (list, tuple)) else [slots])]
    key = _key(pl, len(slots))
    if cache and os.path.exists(cache):
        rec = json.load(open(cache)).get(key)
        if rec:
            pl.set_scatter_policy(rec["regroup_every"], rec["deferred"])
            return (rec["regroup_every"], rec["deferred"]), rec.get("ms_per_iter", {})
    saved = pl.scatter_policy()
    pos = [pl.positions(s) for s in slots]
    scratch = [pl.new_slot() for _ in slots]
    timings = {}
    try:
        for every, deferred in candidates:
            pl.set_scatter_policy(every, deferred)
            runs = []
            for _ in range(repeats):
                for sc, (x, y) in zip(scratch, pos):
                    pl.set_positions(sc, x, y)
                pl.iterate(scratch, gamma, warm, hpwl=True)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                pl.iterate(scratch, gamma, iters, hpwl=True)
                torch.cuda.synchronize()
                runs.append((time.perf_counter() - t0) * 1e3 / iters)
            timings[f"{every},{int(deferred)}"] = sorted(runs)[len(runs) // 2]
    finally:
        for sc in scratch:
            pl.free_slot(sc)
        pl.set_scatter_policy(*saved)
    best = min(timings, key=timings.get)
    every, deferred = int(best.split(",")[0]), best.split(",")[1] == "1"
    pl.set_scatter_policy(every, deferred)
    if cache:
        data = json.load(open(cache)) if os.path.exists(cache) else {}
        data[key] = {"regroup_every": every, "deferred": deferred, "ms_per_iter": timings}
        with open(cache, "w") as fh:
            json.dump(data, fh, indent=1)
    return (every, deferred), timings
