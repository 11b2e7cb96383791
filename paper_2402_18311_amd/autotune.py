"""Timing-based choice of the launch settings of a netlist for a batch of slots: the charge
scatter's grouping policy, then the launch shapes (the net sweep's block order, the Poisson
solve's block width, and whether a rebuilt grouping's accumulation reads charge records).
Results never depend on them beyond the documented last-bit differences of reduced totals;
only speed does.

The scatter groups cells by bin tile and rebuilds the grouping every few evaluations; how
often, and whether the rebuilding evaluation accumulates in the old grouping (one launch
fewer) or the new one (no stale cells), depends on how far cells move per iteration, which
differs between netlists and between the early and late phases of a placement.  tune_scatter
times each candidate on scratch slots that start from the given slots' current positions (the
optimiser restarts there) and keeps the fastest.  A JSON cache keyed by the netlist's shape
and the batch size skips the timing.

    best = tune_scatter(pl, slots, gamma)            # applies and returns (every, deferred)
    shape = tune_launch(pl, slots, gamma)            # applies and returns {tunable: value}
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


# (sweep interleave, spectral threads per block: 0 = by launch size, charge records,
#  non-temporal sweep hints)
LAUNCH_CANDIDATES = tuple((i, t, r, n) for n in (0, 1) for r in (1, 0) for i in (0, 1)
                          for t in (0, 512, 1024))
_LAUNCH_TUNABLES = ("HP_TUNE_SWEEP_INTERLEAVE", "HP_TUNE_SPECTRAL_THREADS", "HP_TUNE_CHARGE_RECORDS",
                    "HP_TUNE_NONTEMPORAL")
_LAUNCH_KEYS = ("interleave", "spectral_threads", "charge_records", "nontemporal")


def tune_launch(pl, slots, gamma, candidates=LAUNCH_CANDIDATES, warm=4, iters=16, repeats=3,
                cache=None):
    """Time the launch-shape candidates as tune_scatter does (scratch slots from the slots'
    positions, median of `repeats`), apply the fastest and return it with the timings."""
    import torch
    from . import hybro as hy
    slots = [int(s) for s in (slots if isinstance(slots, (list, tuple)) else [slots])]
    key = "launch_" + _key(pl, len(slots))
    which = [getattr(hy, n) for n in _LAUNCH_TUNABLES]

    def apply(values):
        for w, v in zip(which, values):
            pl.set_tunable(w, int(v))
    if cache and os.path.exists(cache):
        rec = json.load(open(cache)).get(key)
        if rec and all(k in rec for k in _LAUNCH_KEYS):
            apply([rec[k] for k in _LAUNCH_KEYS])
            return rec, rec.get("ms_per_iter", {})
    saved = [pl.tunable(w) for w in which]
    pos = [pl.positions(s) for s in slots]
    scratch = [pl.new_slot() for _ in slots]
    timings = {}
    try:
        for cand in candidates:
            apply(cand)
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
            timings[",".join(str(int(v)) for v in cand)] = sorted(runs)[len(runs) // 2]
    finally:
        for sc in scratch:
            pl.free_slot(sc)
        apply(saved)
    best = min(timings, key=timings.get)
    values = [int(v) for v in best.split(",")]
    apply(values)
    rec = dict(zip(_LAUNCH_KEYS, values))
    rec["ms_per_iter"] = timings
    if cache:
        data = json.load(open(cache)) if os.path.exists(cache) else {}
        data[key] = rec
        with open(cache, "w") as fh:
            json.dump(data, fh, indent=1)
    return rec, timings
