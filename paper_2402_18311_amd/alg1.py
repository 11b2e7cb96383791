"""Hybro's outer loop (Alg. 1) on the device: place, then repeatedly perturb the best solution,
re-place it and keep the one with the smallest exact HPWL (Eq. 1).

The paper leaves the analytical placer's schedules and stopping rule to the placer it builds
on (Sec. 3.1).  This driver uses the ePlace-style rules (a reading):
  * the placer runs until the density overflow tau (the D(s) <= eps measure of Eq. 1) is at
    most TAU_STOP and the HPWL has stopped falling (it fell by at most PLATEAU of itself over
    the last CHECK iterations, or rose: past that point the growing penalty only spreads the
    cells further at the cost of wirelength), or for at most `max_iters` iterations;
  * every CHECK iterations the smoothing of Eq. 3 follows the overflow,
        gamma(tau) = GAMMA_BINS * bin * 10^((20/9) tau - 11/9),
    and the penalty weight of Eq. 2 is multiplied at every following step by
        mu = clamp(MU_MAX^(1 - dH / (DH_REF * H)), MU_MIN, MU_MAX),
    with dH the HPWL change per iteration over the last CHECK iterations and H the HPWL before
    them; lambda_0 is derived at the first evaluation (scale x |grad WL|_1 / |grad N|_1);
  * the decisions read only the exact integer HPWL and overflow numerator.

Perturbations (Sec. 4.2): Gaussian moves of a fraction of the cells, Shuffle (all) of a
fraction, Shuffle of a fraction of the macros or WireMask over all of them (netlists with
movable macros), or a uniform random restart (the Multiple-restart baseline).  With filler cells (a target density below 1)
the perturbations other than the restart select among the real cells, and the stopping rule
reads the real cells' overflow.  Every iteration runs
on the device (hp_iterate); the host reads two integers every CHECK iterations.

    python -m paper_2402_18311_amd.alg1 --workload mid --rounds 5
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import hybro as hy
from . import netgen

CHECK = 10
TAU_STOP = 0.10
PLATEAU = 1e-3
GAMMA_BINS = 4.0
MU_MAX, MU_MIN = 1.05, 0.95
DH_REF = 3.5e-3
LAMBDA0_SCALE = 1e-4

MODES = {"gauss": hy.HP_PERTURB_GAUSS, "shuffle": hy.HP_PERTURB_SHUFFLE,
         "shuffle-macros": hy.HP_PERTURB_SHUFFLE, "restart": hy.HP_PERTURB_UNIFORM,
         "wiremask": None}
FRACTIONS = {"gauss": 0.05, "shuffle": 0.5, "shuffle-macros": 0.5, "restart": 1.0,
             "wiremask": 1.0}


def gamma_of(tau: float, bin_w: float) -> float:
    return GAMMA_BINS * bin_w * 10.0 ** ((20.0 / 9.0) * tau - 11.0 / 9.0)


def mu_of(h: int, h_prev: int) -> float:
    d = (h - h_prev) / CHECK
    m = MU_MAX ** (1.0 - d / (DH_REF * h_prev)) if h_prev > 0 else MU_MAX
    return min(MU_MAX, max(MU_MIN, m))


def _tau(pl, slot: int, st=None) -> float:
    """Overflow at the slot's evaluation point; with filler cells, that of the real cells."""
    if getattr(pl.nl, "n_fillers", 0):
        return float(pl.overflow_of_cells(slot)[1])
    return float((st or pl.state(slot))["overflow"])


def global_place(pl, slot: int, max_iters: int) -> dict:
    """One run of the placer from the slot's current positions: returns iterations, the final
    HPWL_q of u and the final overflow (of the real cells when the netlist has fillers)."""
    nl = pl.nl
    pl.eval(slot, gamma_of(1.0, nl.bin_w), lam=0.0)  # overflow at the start
    tau = _tau(pl, slot)
    h_prev = int(pl.hpwl(slot)[0])
    hy.hp_set_lambda_ratio(pl.ctx, slot, MU_MAX)
    k = 0
    settled = False
    while k < max_iters and not (tau <= TAU_STOP and settled):
        n = min(CHECK, max_iters - k)
        pl.iterate(slot, gamma_of(tau, nl.bin_w), n, hpwl=True)
        k += n
        st = pl.state(slot)
        tau = _tau(pl, slot, st)
        h = int(st["hpwl_q"])
        settled = h - h_prev >= -PLATEAU * h_prev
        hy.hp_set_lambda_ratio(pl.ctx, slot, mu_of(h, h_prev))
        h_prev = h
    return {"iters": k, "hpwl_q": h_prev, "overflow": tau}


def hybro(pl, rounds: int, mode: str = "gauss", fraction: float = 0.05, sigma_bins: float = 8.0,
          seed: int = 0, max_iters: int = 1000, x0=None, y0=None,
          backtracking: bool = False) -> dict:
    """Alg. 1: the incumbent is the placement of (x0, y0); each round perturbs it (`mode`),
    re-places and keeps the better.  With `backtracking` the placer's Nesterov steps are
    checked and redone as in ePlace.  Returns the per-round trace."""
    nl = pl.nl
    inc, work = pl.new_slot(), pl.new_slot()
    try:
        pl.set_positions(inc, nl.x0 if x0 is None else x0, nl.y0 if y0 is None else y0)
        pl.set_schedule(inc, LAMBDA0_SCALE, 4.0, 1000)
        pl.set_schedule(work, LAMBDA0_SCALE, 4.0, 1000)
        pl.set_backtracking(inc, backtracking)
        pl.set_backtracking(work, backtracking)
        first = global_place(pl, inc, max_iters)
        best = first["hpwl_q"]
        trace = [{"round": 0, **first, "best_hpwl_q": best}]
        import torch
        ix = torch.empty(nl.n_movable, dtype=pl.tdtype, device=pl.dev)
        iy = torch.empty_like(ix)
        for r in range(rounds):
            hy.hp_get_positions(pl.ctx, inc, ix, iy, True)
            pl.set_positions(work, ix, iy)
            if mode == "wiremask":  # every macro, largest first (no fraction, no seed)
                pl.wiremask(work)
            else:
                pool = nl.macros if mode == "shuffle-macros" else None
                if pool is None and getattr(nl, "n_fillers", 0) and mode != "restart":
                    pool = np.arange(nl.n_movable - nl.n_fillers, dtype=np.int32)  # real cells
                pl.perturb(work, MODES[mode], fraction, sigma_bins, seed + r, want_idx=False,
                           cells=pool)
            res = global_place(pl, work, max_iters)
            won = pl.select_best([work], inc)
            best = min(best, res["hpwl_q"])
            trace.append({"round": r + 1, **res, "kept": bool(won >= 0), "best_hpwl_q": best})
        return {"mode": mode, "rounds": rounds, "best_hpwl_q": best, "trace": trace}
    finally:
        pl.free_slot(inc)
        pl.free_slot(work)


def main():
    ap = argparse.ArgumentParser(description="Hybro (Alg. 1) against Multiple-restart")
    ap.add_argument("--workload", default="mid")
    ap.add_argument("--rounds", type=int, default=5)
    ap.add_argument("--max-iters", type=int, default=1000)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--modes", default="gauss,shuffle,restart")
    ap.add_argument("--backtracking", action="store_true",
                    help="ePlace backtracking of the placer's Nesterov steps")
    ap.add_argument("--target-density", type=float, default=1.0,
                    help="below 1: add filler cells and stop on the real cells' overflow")
    a = ap.parse_args()
    nl = netgen.make_netlist(a.workload, a.seed)
    if a.target_density < 1.0:
        nl = netgen.with_fillers(nl, a.target_density, a.seed)
    pl = hy.Placer(nl, precision=32, target_density=a.target_density)
    out = {"workload": a.workload, "rounds": a.rounds, "max_iters": a.max_iters,
           "backtracking": a.backtracking, "target_density": a.target_density,
           "fillers": nl.n_fillers, "runs": []}
    for mode in a.modes.split(","):
        if mode in ("shuffle-macros", "wiremask") and nl.macros is None:
            raise SystemExit(f"{a.workload} has no movable macros (try mid_mm)")
        frac = FRACTIONS[mode]
        t0 = time.perf_counter()
        r = hybro(pl, a.rounds, mode, frac, 8.0, a.seed, a.max_iters,
                  backtracking=a.backtracking)
        r["seconds"] = round(time.perf_counter() - t0, 3)
        r["gp_iterations"] = sum(t["iters"] for t in r["trace"])
        out["runs"].append(r)
        print(f"{mode:8s} best HPWL {r['best_hpwl_q'] / 65536:.1f}  "
              f"({r['gp_iterations']} iterations, {r['seconds']} s)", flush=True)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
