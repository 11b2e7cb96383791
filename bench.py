"""Benchmark of the placer hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload mid] [--no-cpu-baseline]

Workload: the "mid" synthetic netlist (210,000 movable unit-height cells, 500 fixed macros on
20% of the die, 220,000 nets with 0.1% of 200-2000 pins, 512 x 512 bins, FP32), shaped like
the adaptec1 design of Table 1.  One step is one iteration of the placer: the objective and
gradient of Eq. 2 (WA wirelength of Eq. 3, charge scatter, Poisson solve, field gather), the
preconditioned Nesterov step, and the exact HPWL of Eq. 1 with the overflow.  The untimed
warmup places the netlist from random positions (W iterations) to give the incumbent; the
timed region is one Hybro round (Alg. 1) on it: perturb the incumbent (Gaussian, 5% of the
cells, sigma = 8 bins), K placer iterations, then keep the better of the result and the
incumbent.

Prints one JSON line: iterations/s, per-step milliseconds, the roofline of the dominant kernel
(algorithmic bytes / its average duration from HIP events recorded around every launch in the
timed region) and the CPU oracle's rate on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Sources that define the first launch of an evaluation (the dominant kernel); the stored HBM
# traffic is used only while their hash matches the one it was measured with.
FRONT_SOURCES = ["paper_2402_18311_amd/csrc/k_sweep.hip", "paper_2402_18311_amd/csrc/hp_binning.h",
                 "paper_2402_18311_amd/csrc/hp_device.h", "paper_2402_18311_amd/csrc/hp_internal.h"]
TRAFFIC_FILE = os.path.join("profiles", "eval_front_kernel_mid_traffic.json")
CALIB_BYTES = 256 << 20  # the calibration copy: 256 MiB read and 256 MiB written
METRIC = ("placer iters/sec + HBM GB/s; batched-vs-plain restarts/sec, p50/p99 at equal HPWL")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(nl, rs=4):
    """Compulsory bytes each kernel must move per launch (each input read once, each output
    written once), for one slot.  Intermediates count for the kernel that produces or consumes
    them."""
    deg = np.diff(nl.net_start)
    E2 = int(np.sum(deg >= 2))
    P2 = int(np.sum(deg[deg >= 2]))
    N, Nall = nl.n_movable, nl.n_cells
    Pm = int(np.sum(nl.pin_cell[np.repeat(deg >= 2, deg)] < N))
    M2 = nl.mx * nl.my
    wa = 4 * (E2 + 1) + 4 * P2 + 2 * rs * P2 + 2 * rs * Nall + 2 * rs * P2
    hpwl = 4 * (E2 + 1) + 4 * P2 + 8 * P2 + 2 * rs * Nall
    scatter = 2 * rs * N + 20 * N + 8 * M2
    return {
        # the first launch of an evaluation: WA sweep of v (net_start, pin cell ids, pin
        # offsets, every position once, pin gradients out), HPWL sweep of u (quantized offsets,
        # u; the topology is shared), and the charge scatter of v (charge constants in, the
        # int64 map out; v already counted); the grouping and tile windows are intermediates
        "eval_front_kernel": wa + (8 * P2 + 2 * rs * Nall) + (20 * N + 8 * M2),
        "sweep_wa": wa,
        "sweep_hpwl": hpwl,
        "bin_accum_kernel": scatter,
        # cell CSR, pin gradients, positions, charge constants, the field map, gradient out;
        # for the next step's reductions also v_prev, g_prev and the preconditioner's inputs
        "cell_grad_kernel": 4 * (N + 1) + 4 * Pm + 2 * rs * Pm + 2 * rs * N + 20 * N
        + 2 * rs * M2 + 2 * rs * N + 3 * 2 * rs * N,
        # fixed int64 map in, row transform out (the movable map is the scatter's output)
        "spec_rows_fwd": 8 * M2 + rs * M2,
        "spec_cols": rs * M2 + 2 * rs * M2,
        "spec_rows_inv": 2 * rs * M2 + 2 * rs * M2,
        # v, v_prev, g, g_prev, pins + area
        "step_norms_kernel": 4 * 2 * rs * N + 2 * rs * N,
        # pins, area, clamp bounds, v, u, g in; u, v, v_prev, g_prev out
        "step_update_kernel": 4 * rs * N + 3 * 2 * rs * N + 4 * 2 * rs * N,
    }


def cpu_baseline(nl, gamma, budget_s=15.0, max_iters=400):
    """The FP64 oracle, as it stands, on a bounded sample of the same workload: whole placer
    iterations (objective + gradient, Nesterov step, exact HPWL) from the initial positions."""
    from oracle import oracle as O
    o = O.Oracle(nl)
    n = nl.n_movable
    st = o.new_state(nl.x0, nl.y0)
    ratio = o.lambda_ratio(4.0, 1000)
    lam = None
    t0 = time.perf_counter()
    it = 0
    while it < max_iters:
        r = o.eval(st["v"][:n], st["v"][n:], gamma)
        gw = np.concatenate([r["gwx"], r["gwy"]])
        gd = np.concatenate([r["gdx"], r["gdy"]])
        lam = 1e-4 * np.abs(gw).sum() / np.abs(gd).sum() if lam is None else lam * ratio
        o.nesterov_step(lam, gw + lam * gd, st)
        o.hpwl_q(st["u"][:n], st["u"][n:])
        it += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": it / dt, "unit": "iter/s", "cores": O.num_threads(), "kind": "oracle",
            "sample": f"{it} placer iterations (objective+gradient, Nesterov step, exact HPWL) "
                      f"of the mid workload from its initial placement, FP64, {dt:.1f} s"}


def sources_hash(files=FRONT_SOURCES):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def pmc_summary(fetch_dir, write_dir, kernel="eval_front_kernel", last=None):
    """Per-launch HBM traffic of `kernel` from two rocprofv3 --pmc runs (FETCH_SIZE, then
    WRITE_SIZE, KiB per dispatch), each scaled by what the same counter reads for the 256 MiB
    calibration copy of the same run (--copy-calibration).  With `last`, the average is over
    the kernel's last `last` dispatches (the timed round of the profiled run) and the average
    over all of them is recorded beside it.  Writes TRAFFIC_FILE."""
    import csv
    import glob

    def load(d, counter):
        f = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)[0]
        vals, calib = [], []
        for r in csv.DictReader(open(f)):
            if r["Counter_Name"] != counter:
                continue
            v = float(r["Counter_Value"])
            if kernel in r["Kernel_Name"]:
                vals.append((int(r.get("Dispatch_Id") or r.get("Correlation_Id") or 0), v))
            elif "copyBuffer" in r["Kernel_Name"]:
                calib.append(v)
        vals = [v for _, v in sorted(vals)]
        tail = vals[-last:] if last else vals
        return sum(tail) / len(tail), max(calib), len(tail), sum(vals) / len(vals)

    fe, fc, n1, fe_all = load(fetch_dir, "FETCH_SIZE")
    wr, wc, n2, wr_all = load(write_dir, "WRITE_SIZE")
    kib = CALIB_BYTES / 1024
    ff, wf = kib / fc, kib / wc
    traffic = (fe * ff + wr * wf) * 1024
    rec = {"kernel": kernel, "workload": "mid", "fetch_kib_per_launch": round(fe, 1),
           "write_kib_per_launch": round(wr, 1), "launches": [n1, n2],
           "all_launches_fetch_write_kib": [round(fe_all, 1), round(wr_all, 1)],
           "calibration_copy_kib": [round(fc, 1), round(wc, 1)],
           "fetch_factor": round(ff, 4), "write_factor": round(wf, 4),
           "traffic_bytes_per_launch": int(traffic), "sources_hash": sources_hash()}
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(os.path.join(ROOT, TRAFFIC_FILE), "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec))


def stored_traffic(kernel):
    """HBM bytes per launch of `kernel` measured by counters, or None if absent or stale."""
    path = os.path.join(ROOT, TRAFFIC_FILE)
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel") != kernel or rec.get("sources_hash") != sources_hash():
        return None
    return rec["traffic_bytes_per_launch"]


def batched_round(pl, hy, nl, gamma, inc, K, T, seed0):
    """One batched Hybro round (K perturbed restarts of the incumbent, each Gaussian 5%,
    sigma 8 bins, then T iterations) as one K-slot launch sequence, against the same K
    restarts solved one slot at a time.  Returns restarts/s of both and whether every
    restart's final HPWL_q agrees bit for bit."""
    import torch
    ix = torch.empty(nl.n_movable, dtype=torch.float32, device="cuda")
    iy = torch.empty_like(ix)
    hy.hp_get_positions(pl.ctx, inc, ix, iy, True)
    res = {}
    for mode in ("plain", "batched"):
        slots = [pl.new_slot() for _ in range(K)]
        for s in slots:
            pl.set_positions(s, ix, iy)
            pl.set_schedule(s, 1e-4, 4.0, T)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k, s in enumerate(slots):
            pl.perturb(s, hy.HP_PERTURB_GAUSS, 0.05, 8.0, seed0 + k, want_idx=False)
            if mode == "plain":
                pl.iterate(s, gamma, T, hpwl=True)
        if mode == "batched":
            pl.iterate(slots, gamma, T, hpwl=True)
        q = pl.hpwl(slots)  # reduces the last sweeps (synchronises)
        dt = time.perf_counter() - t0
        res[mode] = (K / dt, dt, [int(v) for v in q])
        for s in slots:
            pl.free_slot(s)
    return {"restarts": K, "iterations": T,
            "batched_restarts_per_s": round(res["batched"][0], 3),
            "plain_restarts_per_s": round(res["plain"][0], 3),
            "speedup": round(res["batched"][0] / res["plain"][0], 3),
            "batched_round_s": round(res["batched"][1], 4),
            "plain_rounds_s": round(res["plain"][1], 4),
            "equal_hpwl": res["batched"][2] == res["plain"][2],
            "best_hpwl": min(res["batched"][2]) / 65536}


def large_run(hy, netgen, seed, warm, steps):
    """Plain-method iterations on the large synthetic netlist (2.2 M cells, 1024 x 1024 bins,
    FP32 with the int64 charge map): iterations/s over `steps` iterations after `warm`, and the
    first launch's HBM rate from HIP events on its launches in that timed region."""
    import torch
    nl = netgen.make_netlist("large", seed)
    pl = hy.Placer(nl, precision=32)
    g = 4 * nl.bin_w
    s = pl.new_slot()
    pl.set_positions(s, nl.x0, nl.y0)
    pl.set_schedule(s, 1e-4, 4.0, warm + steps)
    pl.iterate(s, g, warm, hpwl=True)
    from paper_2402_18311_amd import autotune
    policy, _ = autotune.tune_scatter(pl, [s], g)  # untimed; scratch slots from s's positions
    hy.hp_profile_enable(pl.ctx, True, "eval_front_kernel")
    hy.hp_profile_read(pl.ctx, reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pl.iterate(s, g, steps, hpwl=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = hy.hp_profile_read(pl.ctx, reset=True)
    hy.hp_profile_enable(pl.ctx, False)
    c, ms = prof.get("eval_front_kernel", (0, 0.0))
    ab = algorithmic_bytes(nl)["eval_front_kernel"]
    avg = ms * 1e-3 / max(c, 1)
    hq = pl.hpwl(s)[0]
    out = {"workload": f"large: {nl.n_movable} movable cells, {nl.n_fixed} fixed macros, "
                       f"{nl.n_nets} nets / {nl.n_pins} pins, {nl.mx}x{nl.my} bins, FP32, "
                       f"int64 charge map",
           "iter_per_s": round(steps / dt, 2), "ms_per_step": round(1e3 * dt / steps, 4),
           "steps": steps, "warmup": warm, "hpwl": hq / 65536,
           "scatter_policy": {"regroup_every": policy[0], "deferred": policy[1]},
           "front_kernel_avg_us": round(avg * 1e6, 3),
           "front_kernel_gbs": round(ab / avg / 1e9, 1) if c else None,
           "front_kernel_frac": round(ab / avg / 1e9 / HBM_PEAK_GBS, 4) if c else None}
    pl.close()
    return out


def macros_run(hy, netgen, seed, warm, steps):
    """The mid netlist with its 500 macros movable (mixed-size placement; the macros take the
    block-per-cell charge path): iterations/s over `steps` plain-method iterations after
    `warm`, then one Hybro-Shuffle round (half of the macros exchange places, Sec. 4.2, and
    `steps` iterations follow) and one WireMask pass over all macros, each timed on its own."""
    import torch
    nl = netgen.make_netlist("mid_mm", seed)
    pl = hy.Placer(nl, precision=32)
    g = 4 * nl.bin_w
    s = pl.new_slot()
    pl.set_positions(s, nl.x0, nl.y0)
    pl.set_schedule(s, 1e-4, 4.0, warm + steps)
    pl.iterate(s, g, warm, hpwl=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pl.iterate(s, g, steps, hpwl=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    h0 = pl.hpwl(s)[0]
    w = pl.new_slot()
    ix = torch.empty(nl.n_movable, dtype=torch.float32, device="cuda")
    iy = torch.empty_like(ix)
    hy.hp_get_positions(pl.ctx, s, ix, iy, True)
    pl.set_positions(w, ix, iy)
    pl.set_schedule(w, 1e-4, 4.0, steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    moved = pl.perturb(w, hy.HP_PERTURB_SHUFFLE, 0.5, 0.0, 0x5EED, want_idx=False,
                       cells=nl.macros)
    pl.iterate(w, g, steps, hpwl=True)
    h1 = pl.hpwl(w)[0]  # synchronises
    dr = time.perf_counter() - t1
    # one WireMask pass (Sec. 4.2) over every macro of the same placement, largest first
    pl.set_positions(w, ix, iy)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    wm_moved = pl.wiremask(w)  # synchronises
    dw = time.perf_counter() - t2
    h2 = pl.hpwl(w)[0]
    out = {"workload": f"mid_mm: {nl.n_movable} movable cells of which {len(nl.macros)} macros, "
                       f"{nl.n_nets} nets / {nl.n_pins} pins, {nl.mx}x{nl.my} bins, FP32",
           "iter_per_s": round(steps / dt, 2), "ms_per_step": round(1e3 * dt / steps, 4),
           "steps": steps, "warmup": warm, "hpwl": h0 / 65536,
           "shuffle_round": {"macros_moved": int(moved), "iterations": steps,
                             "seconds": round(dr, 4), "hpwl": h1 / 65536},
           "wiremask_pass": {"macros": len(nl.macros), "macros_moved": int(wm_moved),
                             "seconds": round(dw, 4), "hpwl_before": h0 / 65536,
                             "hpwl_after": h2 / 65536}}
    pl.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=1000,
                    help="untimed iterations that place the incumbent (a full placement run)")
    ap.add_argument("--workload", default="mid")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true",
                    help="time without the per-launch events (no roofline)")
    ap.add_argument("--large-steps", type=int, default=500,
                    help="timed iterations on the large netlist (0 skips it)")
    ap.add_argument("--macro-steps", type=int, default=1000,
                    help="timed iterations on mid with movable macros (0 skips it)")
    ap.add_argument("--serve-jobs", type=int, default=16,
                    help="jobs of the serving-mix trace (0 skips it)")
    ap.add_argument("--batch", type=int, default=32,
                    help="restarts of the batched-round measurement (0 skips it)")
    ap.add_argument("--pmc-last", type=int, default=None,
                    help="with --pmc-summary: average the kernel's last N dispatches only")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="reduce two rocprofv3 --pmc output folders to the stored traffic "
                         "record and exit")
    ap.add_argument("--scatter-policy", metavar="EVERY,DEFERRED",
                    help="use this charge-scatter policy (e.g. 8,1) instead of timing the "
                         "candidates before the round")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the round, copy 256 MiB device-to-device once: the reference "
                         "dispatch for scaling hardware byte counters")
    args = ap.parse_args()
    if args.pmc_summary:
        pmc_summary(*args.pmc_summary, last=args.pmc_last)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the placer runs on a single MI355X; "
              "--gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2402_18311_amd import hybro as hy
    from paper_2402_18311_amd import netgen
    if not os.path.exists(hy.LIB_PATH):
        from paper_2402_18311_amd import build as b
        b.build()

    nl = netgen.make_netlist(args.workload, args.seed)
    gamma = 4 * nl.bin_w
    K, W = args.steps, args.warmup
    pl = hy.Placer(nl, precision=32)
    work, inc = pl.new_slot(), pl.new_slot()

    def round_(iters, seed):
        """One Hybro round on `work`: perturb, iters placer iterations (objective + gradient,
        Nesterov step, exact HPWL; one library call), keep the best."""
        pl.perturb(work, hy.HP_PERTURB_GAUSS, 0.05, 8.0, seed, want_idx=False)
        pl.iterate(work, gamma, iters, hpwl=True)
        pl.select_best([work], inc, want_host=False)

    def restart_from_incumbent(iters):
        ix = torch.empty(nl.n_movable, dtype=torch.float32, device="cuda")
        iy = torch.empty_like(ix)
        hy.hp_get_positions(pl.ctx, inc, ix, iy, True)
        pl.set_positions(work, ix, iy)
        pl.set_schedule(work, 1e-4, 4.0, iters)

    log(f"[bench] {nl.name}: {nl.n_movable} movable, {nl.n_fixed} fixed, {nl.n_nets} nets, "
        f"{nl.n_pins} pins, {nl.mx}x{nl.my} bins; warmup {W}, steps {K}")
    # every kernel once (code objects load lazily on first launch), then the incumbent: a full
    # placement from the random initial positions
    pl.set_positions(work, nl.x0, nl.y0)
    pl.perturb(work, hy.HP_PERTURB_SHUFFLE, 0.5, 0.0, 1, want_idx=False)
    pl.perturb(work, hy.HP_PERTURB_GAUSS, 0.5, 8.0, 2, want_idx=False)
    pl.set_positions(work, nl.x0, nl.y0)
    pl.set_schedule(work, 1e-4, 4.0, max(W, 1))
    pl.iterate(work, gamma, W, hpwl=True)
    pl.hpwl(work)
    pl.select_best([work], inc)
    torch.cuda.synchronize()
    log("[bench] warmup done")

    # the scatter's grouping policy, chosen by timing (untimed) from the state the timed round
    # starts in: the incumbent with a Gaussian perturbation
    if args.scatter_policy:
        e, d = (int(v) for v in args.scatter_policy.split(","))
        pl.set_scatter_policy(e, bool(d))
        policy, tune_ms = pl.scatter_policy(), {}
    else:
        from paper_2402_18311_amd import autotune
        restart_from_incumbent(K)
        pl.perturb(work, hy.HP_PERTURB_GAUSS, 0.05, 8.0, 0x7E57, want_idx=False)
        policy, tune_ms = autotune.tune_scatter(pl, [work], gamma)
    log(f"[bench] scatter policy {policy} ({tune_ms})")

    # kernel table: a short round with every launch bracketed by events
    prof = {}
    if not args.no_profile:
        P = min(K, 200)
        restart_from_incumbent(P)
        hy.hp_profile_enable(pl.ctx, True)
        hy.hp_profile_read(pl.ctx, reset=True)
        round_(P, 0xBEEF)
        prof = hy.hp_profile_read(pl.ctx, reset=True)
        hy.hp_profile_enable(pl.ctx, False)
    ab = algorithmic_bytes(nl)
    kernels = {k: {"launches": c, "avg_us": 1e3 * ms / max(c, 1), "total_ms": ms}
               for k, (c, ms) in sorted(prof.items(), key=lambda kv: -kv[1][1])}
    dom = next((k for k in kernels if k in ab), None)

    # the timed round; only the dominant kernel's launches carry events
    restart_from_incumbent(K)
    if dom:
        hy.hp_profile_enable(pl.ctx, True, dom)
        hy.hp_profile_read(pl.ctx, reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    round_(K, 0xC0FFEE)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    live = {}
    if dom:
        live = hy.hp_profile_read(pl.ctx, reset=True)
        hy.hp_profile_enable(pl.ctx, False)
    final = pl.state(inc)
    log(f"[bench] timed {K} iterations in {dt:.3f} s; incumbent HPWL "
        f"{final['hpwl_q'] / 65536:.1f}")
    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")  # 256 MiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    roof = None
    if dom and dom in live:
        c, ms = live[dom]
        avg_s = ms * 1e-3 / max(c, 1)
        achieved = ab[dom] / avg_s / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": stored_traffic(dom),
                "kernel": dom, "algorithmic_bytes": int(ab[dom]), "launches": c,
                "avg_us": round(avg_s * 1e6, 3)}
    for k, v in kernels.items():
        if k in ab:
            v["algorithmic_gbs"] = round(ab[k] / (v["avg_us"] * 1e-6) / 1e9, 1)
    it_bytes = sum(ab[k] for k in ("eval_front_kernel", "cell_grad_kernel", "spec_rows_fwd",
                                   "spec_cols", "spec_rows_inv", "step_update_kernel"))
    ms_step = 1e3 * dt / K
    out = {
        "metric": METRIC, "value": round(K / dt, 2), "unit": "iter/s", "n_gpus": 1, "steps": K,
        "warmup": W, "ms_per_step": round(ms_step, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{nl.name}: {nl.n_movable} movable cells, {nl.n_fixed} fixed "
                               f"macros (20% of die), {nl.n_nets} nets / {nl.n_pins} pins, "
                               f"{nl.mx}x{nl.my} bins, gamma = 4 bins, one Hybro round "
                               f"(Gaussian perturb 5%, sigma 8 bins) of {K} iterations",
                   "global_batch": 1, "parallelism": "single-gpu"},
        "hbm_gbps_algorithmic": round(it_bytes / (ms_step * 1e-3) / 1e9, 1),
        "timing": ("value: wall clock of the timed round, GPU synchronised on both sides; "
                   "roofline: HIP events around every launch of the dominant kernel in that "
                   "round; kernels: a separate 200-iteration round with events on every launch"),
        "final_hpwl": final["hpwl_q"] / 65536,
        "tuning": {"scatter_policy": {"regroup_every": policy[0], "deferred": policy[1]},
                   "ms_per_iter": {k: round(v, 4) for k, v in tune_ms.items()}},
        "roofline": roof,
        "kernels": {k: {kk: (round(vv, 3) if isinstance(vv, float) else vv)
                        for kk, vv in v.items()} for k, v in kernels.items()},
    }
    if args.batch > 0:
        log(f"[bench] batched round: {args.batch} restarts x {K} iterations, batched vs plain")
        out["batched"] = batched_round(pl, hy, nl, gamma, inc, args.batch, K, 0xB00)
    if args.large_steps > 0:
        log(f"[bench] large netlist: 300 + {args.large_steps} iterations")
        out["large"] = large_run(hy, netgen, args.seed, 300, args.large_steps)
    if args.macro_steps > 0:
        log(f"[bench] movable macros: 600 + {args.macro_steps} iterations, one shuffle round")
        out["movable_macros"] = macros_run(hy, netgen, args.seed, 600, args.macro_steps)
    if args.serve_jobs > 0:
        from paper_2402_18311_amd import serve
        log(f"[bench] serving mix: {args.serve_jobs} jobs, 10 k - 2.2 M cells, 500 iterations")
        out["serving"] = serve.measure(args.serve_jobs, 10_000, 2_200_000, 500, 8.0, 0.8,
                                       args.seed, log=log)
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample ...")
        out["cpu_baseline"] = cpu_baseline(nl, gamma)
    pl.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
